// Crest-factor search for tone phases on the device (plan time).
//
// The tone phases theta_k set the peak (crest) factor of the static waveform
// (Theory section: the paper keeps it low with phases after Schroeder 1970).
// The closed forms (Schroeder's rule, Newman's phases; phases.cpp) are made for
// evenly spaced tones; on irregular bins they leave the crest factor at the
// level of random phases. awg_phase_search minimises the crest factor of one
// period of y[n] = sum_k A_k sin(2 pi b_k n / L + theta_k) directly, by the
// Chebyshev approach of Guillaume, Schoukens, Pintelon and Kollar (1991):
// minimise the l_p norm of y over the period for growing even p, which tends to
// the peak, each stage by L-BFGS from the previous stage's phases. With
// g_n = sign(y_n) |y_n|^(p-1),
//     F = (1/p) log sum_n |y_n|^p,   dF/dtheta_k = A_k sum_n g_n cos(2 pi b_k n / L + theta_k) / sum_n |y_n|^p.
// Per evaluation the device computes y over the period (exact phase words, as
// the direct kernel), its peak, the normalised powers and g, and the gradient
// correlations (one cosine per tone-sample); the host keeps the L-BFGS state.
// It starts from the better closed form and returns the phases with the lowest
// crest factor seen, measured as max|y| / sqrt(sum A^2 / 2) on the phases as a
// plan would take them (phase words nint(turns 2^64)).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "awg_internal.h"

namespace awg {

namespace {

struct SearchTone {
    uint64_t p, f;       // phase and frequency words (exact)
    float a;             // amplitude
    float pad;
};

constexpr int kSynthPerThread = 16;                 // samples per thread (synthesis, powers)
constexpr uint64_t kSynthBlock = 256 * kSynthPerThread;
constexpr int kCorrPerThread = 64;                  // samples per thread (correlations)
constexpr uint64_t kCorrChunk = 256 * kCorrPerThread;
constexpr int kCorrTones = 32;                      // tones per correlation workgroup

__device__ __forceinline__ float word_turn(uint64_t w)
{
    return (float)(int32_t)(uint32_t)(w >> 32) * 0x1p-32f;     // [-1/2, 1/2) turn
}

// y[n] for n in [0, L) (L a multiple of kSynthBlock), and the peak |y| as the
// bit pattern of a non-negative float (atomic max).
__global__ __launch_bounds__(256) void search_synth_kernel(const SearchTone *__restrict__ tones, int32_t K,
                                                           float *__restrict__ y, unsigned *__restrict__ peak_bits)
{
    const uint64_t base = (uint64_t)blockIdx.x * kSynthBlock + (uint64_t)threadIdx.x * kSynthPerThread;
    float acc[kSynthPerThread];
#pragma unroll
    for (int s = 0; s < kSynthPerThread; ++s) acc[s] = 0.0f;
    for (int32_t k = 0; k < K; ++k) {
        const uint64_t F = tones[k].f;
        const float a = tones[k].a;
        uint64_t ph = tones[k].p + F * base;
#pragma unroll
        for (int s = 0; s < kSynthPerThread; ++s) {
            acc[s] = __builtin_fmaf(a, __builtin_amdgcn_sinf(word_turn(ph)), acc[s]);
            ph += F;
        }
    }
    float m = 0.0f;
#pragma unroll
    for (int s = 0; s < kSynthPerThread; ++s) {
        y[base + s] = acc[s];
        m = fmaxf(m, fabsf(acc[s]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(peak_bits, __float_as_uint(m));
}

// v = y / peak (|v| <= 1): y[n] <- g = sign(v) |v|^(p-1); part[block] = sum |v|^p.
__global__ __launch_bounds__(256) void search_power_kernel(float *__restrict__ y, float inv_peak, float pm1,
                                                           float *__restrict__ part)
{
    __shared__ float red[4];
    const uint64_t base = (uint64_t)blockIdx.x * kSynthBlock + (uint64_t)threadIdx.x * kSynthPerThread;
    float sum = 0.0f;
#pragma unroll
    for (int s = 0; s < kSynthPerThread; ++s) {
        const float v = y[base + s] * inv_peak;
        const float av = fminf(fabsf(v), 1.0f);
        const float q = av > 0.0f ? __builtin_amdgcn_exp2f(pm1 * __builtin_amdgcn_logf(av)) : 0.0f;
        y[base + s] = v < 0.0f ? -q : q;
        sum = __builtin_fmaf(q, av, sum);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// part[c * K + k] = sum over chunk c of g[n] cos(2 pi word_k(n) / 2^64); grid
// (L / kCorrChunk, ceil(K / kCorrTones)).
__global__ __launch_bounds__(256) void search_corr_kernel(const SearchTone *__restrict__ tones, int32_t K,
                                                          const float *__restrict__ g, float *__restrict__ part)
{
    __shared__ float red[kCorrTones][4];
    const uint64_t base = (uint64_t)blockIdx.x * kCorrChunk + (uint64_t)threadIdx.x * kCorrPerThread;
    float gv[kCorrPerThread];
#pragma unroll
    for (int s = 0; s < kCorrPerThread; s += 4) {
        const float4 u = *(const float4 *)(g + base + s);
        gv[s] = u.x; gv[s + 1] = u.y; gv[s + 2] = u.z; gv[s + 3] = u.w;
    }
    const int32_t k0 = (int32_t)blockIdx.y * kCorrTones;
    const int wave = threadIdx.x >> 6;
    for (int t = 0; t < kCorrTones; ++t) {
        const int32_t k = k0 + t;
        if (k >= K) break;
        const uint64_t F = tones[k].f;
        uint64_t ph = tones[k].p + F * base;
        float acc = 0.0f;
#pragma unroll
        for (int s = 0; s < kCorrPerThread; ++s) {
            acc = __builtin_fmaf(gv[s], __builtin_amdgcn_cosf(word_turn(ph)), acc);
            ph += F;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) red[t][wave] = acc;
    }
    __syncthreads();
    if (threadIdx.x < kCorrTones) {
        const int32_t k = k0 + (int32_t)threadIdx.x;
        if (k < K) {
            const float (&r)[4] = red[threadIdx.x];
            part[blockIdx.x * (uint64_t)K + (uint64_t)k] = ((r[0] + r[1]) + r[2]) + r[3];
        }
    }
}

// out[k] = sum over chunks c < n_chunks of part[c * K + k], in FP64.
__global__ __launch_bounds__(256) void search_sum_kernel(const float *__restrict__ part, int32_t K, int32_t n_chunks,
                                                         double *__restrict__ out)
{
    const int32_t k = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= K) return;
    double s = 0.0;
    for (int32_t c = 0; c < n_chunks; ++c) s += (double)part[(uint64_t)c * (uint64_t)K + (uint64_t)k];
    out[k] = s;
}

__global__ void search_zero_kernel(unsigned *w) { *w = 0u; }

awg_status hst(hipError_t e)
{
    if (e == hipSuccess) return AWG_OK;
    return e == hipErrorOutOfMemory ? AWG_E_NOMEM : AWG_E_HIP;
}

const double kTwoPi = 6.283185307179586476925286766559;

// Device state of one search: the tones, y / g over the period, the partial sums.
struct Search {
    int32_t K = 0;
    uint64_t L = 0;
    double rms = 0.0;
    std::vector<SearchTone> host;
    std::vector<float> part_host;
    std::vector<double> tmp;
    SearchTone *d_tones = nullptr;
    float *d_y = nullptr, *d_part = nullptr, *d_corr = nullptr;
    double *d_sum = nullptr;
    unsigned *d_peak = nullptr;
    hipStream_t s = nullptr;
    int32_t evals = 0;
    double best_cf = INFINITY;
    std::vector<double> best;       // phases (rad) of best_cf

    ~Search()
    {
        if (s) (void)hipStreamSynchronize(s);
        for (void *q : {(void *)d_tones, (void *)d_y, (void *)d_part, (void *)d_corr, (void *)d_sum, (void *)d_peak})
            if (q) (void)hipFree(q);
        if (s) (void)hipStreamDestroy(s);
    }

    awg_status setup(const std::vector<uint64_t> &fw, const double *amp)
    {
        host.resize(K);
        double p2 = 0.0;
        for (int32_t k = 0; k < K; ++k) {
            host[k].f = fw[k];
            host[k].a = (float)amp[k];
            host[k].pad = 0.0f;
            p2 += amp[k] * amp[k];
        }
        rms = std::sqrt(p2 / 2.0);
        const uint64_t n_blocks = L / kSynthBlock, n_chunks = L / kCorrChunk;
        part_host.resize(n_blocks);
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMalloc(&d_tones, sizeof(SearchTone) * (size_t)K);
        if (e == hipSuccess) e = hipMalloc(&d_y, sizeof(float) * L);
        if (e == hipSuccess) e = hipMalloc(&d_part, sizeof(float) * n_blocks);
        if (e == hipSuccess) e = hipMalloc(&d_corr, sizeof(float) * n_chunks * (uint64_t)K);
        if (e == hipSuccess) e = hipMalloc(&d_sum, sizeof(double) * (size_t)K);
        if (e == hipSuccess) e = hipMalloc(&d_peak, sizeof(unsigned));
        return hst(e);
    }

    // y over the period for phases given in turns (phase words nint(turns 2^64),
    // as a plan makes them); returns its peak |y| in *peak.
    awg_status synth_turns(const double *turns, float *peak)
    {
        for (int32_t k = 0; k < K; ++k) host[k].p = phase_word(turns[k]);
        hipError_t e = hipMemcpyAsync(d_tones, host.data(), sizeof(SearchTone) * (size_t)K, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(search_zero_kernel, dim3(1), dim3(1), 0, s, d_peak);
            hipLaunchKernelGGL(search_synth_kernel, dim3((uint32_t)(L / kSynthBlock)), dim3(256), 0, s,
                               (const SearchTone *)d_tones, K, d_y, d_peak);
            e = hipGetLastError();
        }
        unsigned bits = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&bits, d_peak, sizeof(unsigned), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hst(e);
        float pk;
        std::memcpy(&pk, &bits, sizeof(float));
        *peak = pk;
        return AWG_OK;
    }

    // the same for phases theta in radians
    awg_status synth(const std::vector<double> &theta, float *peak)
    {
        tmp.resize(K);
        for (int32_t k = 0; k < K; ++k) {
            double t = theta[k] / kTwoPi;
            tmp[k] = t - std::floor(t);
        }
        return synth_turns(tmp.data(), peak);
    }

    // F = (1/p) log sum (y / rms)^p and its gradient (rad^-1) at theta.
    awg_status eval(const std::vector<double> &theta, int p, double *F, std::vector<double> *grad)
    {
        float peak = 0.0f;
        awg_status st = synth(theta, &peak);
        if (st != AWG_OK) return st;
        ++evals;
        const double cf = (double)peak / rms;
        if (cf < best_cf) {
            best_cf = cf;
            best = theta;
        }
        if (!(peak > 0.0f)) return AWG_E_INVALID;
        const uint64_t n_blocks = L / kSynthBlock, n_chunks = L / kCorrChunk;
        hipLaunchKernelGGL(search_power_kernel, dim3((uint32_t)n_blocks), dim3(256), 0, s, d_y, 1.0f / peak,
                           (float)(p - 1), d_part);
        hipLaunchKernelGGL(search_corr_kernel, dim3((uint32_t)n_chunks, (uint32_t)((K + kCorrTones - 1) / kCorrTones)),
                           dim3(256), 0, s, (const SearchTone *)d_tones, K, (const float *)d_y, d_corr);
        hipLaunchKernelGGL(search_sum_kernel, dim3((uint32_t)((K + 255) / 256)), dim3(256), 0, s,
                           (const float *)d_corr, K, (int32_t)n_chunks, d_sum);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(part_host.data(), d_part, sizeof(float) * n_blocks, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(grad->data(), d_sum, sizeof(double) * (size_t)K, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hst(e);
        double S = 0.0;
        for (float v : part_host) S += (double)v;
        if (!(S > 0.0)) return AWG_E_INVALID;
        // sum (y/rms)^p = (peak/rms)^p S
        *F = std::log(S) / p + std::log((double)peak / rms);
        const double scale = 1.0 / ((double)peak * S);
        for (int32_t k = 0; k < K; ++k) (*grad)[k] *= (double)host[k].a * scale;
        return AWG_OK;
    }
};

double dot(const std::vector<double> &a, const std::vector<double> &b)
{
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

// L-BFGS (memory m) on F_p from theta, at most max_evals evaluations; a
// backtracking line search with the Armijo condition.
awg_status lbfgs_stage(Search &S, int p, std::vector<double> &theta, int32_t max_evals)
{
    constexpr int kMem = 8;
    const size_t K = theta.size();
    std::vector<std::vector<double>> sv, yv;
    std::vector<double> rho;
    std::vector<double> g(K), g_new(K), d(K), x_new(K), q(K), alpha(kMem);
    double F = 0.0;
    awg_status st = S.eval(theta, p, &F, &g);
    if (st != AWG_OK) return st;
    int32_t used = 1;
    bool first = true;
    while (used < max_evals) {
        // two-loop recursion: d = -H g
        q = g;
        const int m = (int)sv.size();
        for (int i = m - 1; i >= 0; --i) {
            alpha[i] = rho[i] * dot(sv[i], q);
            for (size_t k = 0; k < K; ++k) q[k] -= alpha[i] * yv[i][k];
        }
        double gamma = 1.0;
        if (m > 0) gamma = dot(sv[m - 1], yv[m - 1]) / dot(yv[m - 1], yv[m - 1]);
        for (size_t k = 0; k < K; ++k) q[k] *= gamma;
        for (int i = 0; i < m; ++i) {
            const double b = rho[i] * dot(yv[i], q);
            for (size_t k = 0; k < K; ++k) q[k] += sv[i][k] * (alpha[i] - b);
        }
        for (size_t k = 0; k < K; ++k) d[k] = -q[k];
        double slope = dot(g, d);
        if (!(slope < 0.0)) {                        // not a descent direction: restart on -g
            sv.clear();
            yv.clear();
            rho.clear();
            for (size_t k = 0; k < K; ++k) d[k] = -g[k];
            slope = dot(g, d);
            first = true;
            if (!(slope < 0.0)) break;               // stationary
        }
        double step = 1.0;
        if (first) {
            double gmax = 0.0;
            for (double v : g) gmax = std::max(gmax, std::fabs(v));
            step = gmax > 0.0 ? std::min(1.0, 0.1 / gmax) : 1.0;
        }
        double F_new = 0.0;
        bool ok = false;
        for (int ls = 0; ls < 20 && used < max_evals; ++ls) {
            for (size_t k = 0; k < K; ++k) x_new[k] = theta[k] + step * d[k];
            st = S.eval(x_new, p, &F_new, &g_new);
            if (st != AWG_OK) return st;
            ++used;
            if (F_new <= F + 1e-4 * step * slope) {
                ok = true;
                break;
            }
            step *= 0.5;
        }
        if (!ok) break;
        std::vector<double> sk(K), yk(K);
        for (size_t k = 0; k < K; ++k) {
            sk[k] = x_new[k] - theta[k];
            yk[k] = g_new[k] - g[k];
        }
        const double sy = dot(sk, yk);
        if (sy > 1e-12 * std::sqrt(dot(sk, sk) * dot(yk, yk))) {
            if ((int)sv.size() == kMem) {
                sv.erase(sv.begin());
                yv.erase(yv.begin());
                rho.erase(rho.begin());
            }
            sv.push_back(sk);
            yv.push_back(yk);
            rho.push_back(1.0 / sy);
        }
        theta = x_new;
        g = g_new;
        const double dF = F - F_new;
        F = F_new;
        first = false;
        if (dF < 1e-9 * std::fabs(F)) break;
    }
    return AWG_OK;
}

}  // namespace

}  // namespace awg

using namespace awg;

extern "C" awg_status awg_phase_search(awg_ctx *ctx, double fs_hz, uint32_t period_log2, const double *f_hz,
                                       const double *amplitude, int32_t n_tones, int32_t max_evals,
                                       double *phase_turns_out, double *crest_out, int32_t *method_out)
{
    if (!ctx || !f_hz || !amplitude || !phase_turns_out || n_tones <= 0 || max_evals < 0) return AWG_E_INVALID;
    if (!std::isfinite(fs_hz) || !(fs_hz > 0.0)) return AWG_E_INVALID;
    if (period_log2 < 14 || period_log2 > 26) return AWG_E_UNSUPPORTED;
    if (n_tones > (1 << 20)) return AWG_E_UNSUPPORTED;
    const uint64_t L = 1ull << period_log2;
    if ((L / kCorrChunk) * (uint64_t)n_tones > (1ull << 28)) return AWG_E_UNSUPPORTED;   // partial sums <= 1 GiB
    double total = 0.0;
    for (int32_t k = 0; k < n_tones; ++k) {
        if (!std::isfinite(amplitude[k]) || amplitude[k] < 0.0) return AWG_E_INVALID;
        total += amplitude[k];
    }
    if (!(total > 0.0)) return AWG_E_INVALID;
    std::vector<uint64_t> fw(n_tones);
    for (int32_t k = 0; k < n_tones; ++k) {
        const awg_status st = freq_word(f_hz[k], fs_hz, period_log2, &fw[k]);
        if (st != AWG_OK) return st;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return AWG_E_HIP;
    try {
        Search S;
        S.K = n_tones;
        S.L = L;
        awg_status st = S.setup(fw, amplitude);
        if (st != AWG_OK) return st;
        // the closed forms, measured; the search starts from the better one
        std::vector<double> turns(n_tones), theta(n_tones);
        int32_t best_method = 0;
        double best_cf = INFINITY;
        std::vector<double> best_theta, best_turns;
        for (int32_t m : {AWG_PHASES_SCHROEDER, AWG_PHASES_NEWMAN}) {
            st = awg_phase_plan(m, f_hz, amplitude, n_tones, turns.data());
            if (st != AWG_OK) return st;
            for (int32_t k = 0; k < n_tones; ++k) theta[k] = kTwoPi * turns[k];
            float peak = 0.0f;
            st = S.synth_turns(turns.data(), &peak);
            if (st != AWG_OK) return st;
            const double cf = (double)peak / S.rms;
            if (cf < best_cf) {
                best_cf = cf;
                best_method = m;
                best_theta = theta;
                best_turns = turns;            // returned as the closed form gives them
            }
        }
        if (max_evals > 0) {
            S.best_cf = best_cf;
            S.best = best_theta;
            theta = best_theta;
            // l_p stages p = 8, 16, ..., 256, the evaluations shared out evenly
            const int stages[] = {8, 16, 32, 64, 128, 256};
            const int n_st = 6;
            int32_t left = max_evals;
            for (int i = 0; i < n_st && left > 0; ++i) {
                const int32_t budget = std::max<int32_t>(1, left / (n_st - i));
                const int32_t before = S.evals;
                st = lbfgs_stage(S, stages[i], theta, budget);
                if (st != AWG_OK) return st;
                left -= S.evals - before;
            }
            if (S.best_cf < best_cf) {
                best_cf = S.best_cf;
                best_method = AWG_PHASES_SEARCH;
                best_theta = S.best;
            }
        }
        for (int32_t k = 0; k < n_tones; ++k) {
            if (best_method != AWG_PHASES_SEARCH) {
                phase_turns_out[k] = best_turns[k];
                continue;
            }
            double t = best_theta[k] / kTwoPi;
            t -= std::floor(t);
            if (t >= 1.0) t -= 1.0;
            phase_turns_out[k] = t;
        }
        // the crest factor of the phases as returned (the words a plan makes of them)
        float peak = 0.0f;
        st = S.synth_turns(phase_turns_out, &peak);
        if (st != AWG_OK) return st;
        if (crest_out) *crest_out = (double)peak / S.rms;
        if (method_out) *method_out = best_method;
        return AWG_OK;
    } catch (...) {
        return AWG_E_NOMEM;
    }
}
