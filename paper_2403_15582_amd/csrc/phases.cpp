// Initial tone phases for a low crest factor (host, plan time).
//
// The tone phases theta_j set the peak (crest) factor of the static waveform,
// which must stay low to protect the acousto-optic deflector (Theory section;
// the paper cites Schroeder 1970 and gives no formula). Two closed forms, tones
// ranked by frequency k = 1..K (equal frequencies in input order):
//   Schroeder, for the power spectrum p_l = A_l^2 / sum A^2:
//     theta_k = -2 pi sum_{l<k} (k - l) p_l = -2 pi (k S_k - T_k),
//     S_k = sum_{l<k} p_l, T_k = sum_{l<k} l p_l (running sums, long double);
//   Newman: theta_k = pi (k - 1)^2 / K, exactly ((k - 1)^2 mod 2K) / 2K turns.
// Phases are returned in turns in [0, 1). awg_peak measures what a phase set
// achieves: the peak of the plan's sum over a range, on the device.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "awg_internal.h"

extern "C" awg_status awg_phase_plan(int32_t method, const double *f_hz, const double *amplitude, int32_t n,
                                     double *phase_turns_out)
{
    if (!f_hz || !phase_turns_out || n <= 0) return AWG_E_INVALID;
    if (method != AWG_PHASES_SCHROEDER && method != AWG_PHASES_NEWMAN) return AWG_E_INVALID;
    if (method == AWG_PHASES_SCHROEDER && !amplitude) return AWG_E_INVALID;
    std::vector<int32_t> order;
    try { order.resize(n); } catch (...) { return AWG_E_NOMEM; }
    for (int32_t i = 0; i < n; ++i) {
        if (!std::isfinite(f_hz[i])) return AWG_E_INVALID;
        if (method == AWG_PHASES_SCHROEDER && !(std::isfinite(amplitude[i]) && amplitude[i] >= 0.0))
            return AWG_E_INVALID;
    }
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return f_hz[a] < f_hz[b]; });
    if (method == AWG_PHASES_NEWMAN) {
        const uint64_t two_k = 2ull * (uint64_t)n;
        for (int32_t r = 0; r < n; ++r) {
            const uint64_t km1 = (uint64_t)r;
            phase_turns_out[order[r]] = (double)((km1 * km1) % two_k) / (double)two_k;
        }
        return AWG_OK;
    }
    long double total = 0.0L;
    for (int32_t i = 0; i < n; ++i) total += (long double)amplitude[i] * (long double)amplitude[i];
    if (!(total > 0.0L)) return AWG_E_INVALID;
    long double S = 0.0L, T = 0.0L;                    // sums over ranks l < k
    for (int32_t r = 0; r < n; ++r) {
        const long double k = (long double)(r + 1);
        long double t = -(k * S - T);
        t -= std::floor(t);
        if (t >= 1.0L) t -= 1.0L;
        phase_turns_out[order[r]] = (double)t;
        const long double a = (long double)amplitude[order[r]];
        const long double pl = a * a / total;
        S += pl;
        T += k * pl;
    }
    return AWG_OK;
}
