"""FP64 CPU oracle for the Kalman filter, fixed-interval smoother and MNE.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, calls or
executes anything in this package: only the tests, the entry module's smoke
check and the benchmark's CPU-baseline leg do. It shares no code with the HIP
path (no kernels, headers, helpers or constants); the two meet only in the
seeded input generator, which holds none of the method's arithmetic.

Contents:

* ``kalman``: the textbook recursions in float64 NumPy/SciPy, in the paper's
  order -- the Kalman filter (eqn6 to eqn10 and the covariance update that
  follows eqn10), the fixed-interval smoother (eqn11 to eqn13, read as the
  standard Rauch-Tung-Striebel form), the MNE estimate (eqn5) and the
  parameter set-up of Section 2.4 (x0 and Sigma_w from MNE estimates), and
  the smoothed means alone by the backward information recursion (modified
  Bryson-Frazier), which reaches the means of eqn12 without the gain A_t.
* ``joint``: the same posteriors by brute force, conditioning the joint
  Gaussian of all time steps at once. It pins the recursions.

Every function is pinned by the CPU tests (brute force, closed forms, special
cases, invariants); none is "parity unpinned".
"""
from .kalman import (kf_filter, rts_smooth, mne_solve, kf_update, smoother_gain, init_from_mne,  # noqa: F401
                     bf_smooth_means)
from .joint import joint_posterior, joint_posterior_information  # noqa: F401
