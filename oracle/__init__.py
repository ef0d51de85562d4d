"""FP64 CPU oracle for SSFM / ESSFM digital backpropagation (Secondini et al.,
"Coherent 100G Nonlinear Compensation with Single-Step Digital Backpropagation").

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct numpy code that
defines what the GPU library must compute.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the GPU
library never does, and this package never imports the GPU library.  The two
share only the seeded input generators of `siggen`, which hold none of the
method's arithmetic.

Modules:
  dbp_ref     step operator (Sec. II, Eqs. 1-3), step schedule, whole-signal
              and overlap-and-save (Sec. III) cascades, FIR linear variant
  adjoint     reverse-mode gradient of a real loss through the cascade
  complexity  the real-operation counts of Sec. III and the channel-memory rule
  fit         least-squares fit of the ESSFM coefficients (Sec. IV)
  rxdsp       receiver DSP after backpropagation (Sec. IV): resampling to two samples
              per symbol, butterfly equalizer, carrier-phase recovery, decisions

Parity status: every function is pinned by tests under tests/ against closed
forms, invariants, brute force or numbers printed in the paper, except the
end-to-end EVM of a realistic nonlinear link, for which the paper prints no
value (parity unpinned; only its parts are pinned).
"""
