"""FP64 CPU oracle of the LM bundle-adjustment step (InstantSfM, arXiv 2510.13310).

THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT. Only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` may import it. It shares
no code with the GPU library (``paper_2510_13310_amd``) and never imports it; both read
inputs from the seeded generator in ``scenes/``, which holds no solver arithmetic.

It is a plain, slow, vectorised NumPy/SciPy implementation in float64 of what the GPU path
computes, written from the paper:

* ``geometry``  quaternion / SO(3) / SE(3) helpers (left perturbation);
* ``model``     reprojection residual Eq. (2), depth residual Eq. (6), masked inverse depth
                Eq. (9), stacked depth-weighted residual Eq. (7), Huber, analytic Jacobians;
* ``extract``   dynamic parameter extraction, Eqs. (10)-(15);
* ``lm``        the LM system Eq. (3) with a dense Schur complement and Cholesky, gain
                ratio, Nielsen damping update, scatter of the compact update;
* ``adjoint``   implicit-function adjoint of the converged solution, solved directly;
* ``gp``        depth-constrained global positioning, Eqs. (1), (4), (5), (8): camera centres,
                points and free per-observation scales, pinned scales from valid depth.

Every function is pinned by ``tests/test_oracle_*.py`` against finite differences, library
routines, brute force on tiny inputs, closed forms or exact recovery of noise-free scenes.
"""
from .model import Problem, huber, residuals, jacobians, cost
from .lm import Options, State, lm_step, solve, extract
from .adjoint import adjoint

__all__ = ["Problem", "huber", "residuals", "jacobians", "cost", "Options", "State",
           "lm_step", "solve", "extract", "adjoint"]
