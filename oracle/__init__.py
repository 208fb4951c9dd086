"""Plain FP64 CPU oracle for least-misfit gridding and degridding.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it. It shares no code with the
HIP library: it is written directly from the paper (Ye, Gull, Tan & Nikolic,
"Optimal gridding and degridding in radio interferometry imaging",
MNRAS 2019), slowly and in double precision, so that it can be checked
against the paper by eye.

Modules
-------
``lmtable``  least-misfit gridding/correcting functions: the normal
             equations (Sec. 2.1, Eqs. 17-19), the Levenberg-Marquardt
             optimisation of h (App. A), the B-matrix least-squares form
             (App. B), look-up table generation (App. E) and
             nearest/Newton interpolation (App. F), the optimal correction
             (Sec. 2.1, Eqs. 12-15) and the map error function (Eqs. 10-11,
             16).
``imaging``  direct gridding (Eqs. 5-6), a hand-written radix-2 FFT,
             correction and cropping (Eq. 4), the prediction path and
             degridding (Sec. 5), and the ground truth: the DFT dirty image
             (Eq. 3) and the direct prediction (Eq. 2), plus the per-pixel
             Cauchy-Schwarz bound (Eqs. 7-8).

Every function is pinned by a ``-m "not gpu"`` test against something the
paper or mathematics fixes (closed forms, identities, printed values,
library routines, brute force); see the test files named in each docstring.
"""
