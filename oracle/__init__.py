"""CPU oracle for multi-tone additive synthesis.

TEST INFRASTRUCTURE. This package is a plain, slow, independent statement of
what the synthesis computes, written from the paper's Theory section
(Eqs. (1)-(8)). Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product library never does, and the two
share no code.

Modules:
  words  -- exact-integer phase and frequency words (Python ``Fraction`` / big
            integers), ramp tables, the piecewise phase definition, and a
            pure-Python evaluator for small cases.
  csynth -- FP64 direct sum over tones and samples in plain C (``synth.c``),
            built with gcc, called through ctypes.

Every function cites the passage it follows. Where a function has no external
pin it says "parity unpinned" in its docstring.
"""
