"""Plain, slow FP64 CPU oracle of the G-ICP tracking path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, helpers or tables); the two meet only in the
seeded input generators of the ``synth`` package.

What it computes, following the paper "RGBD GS-ICP SLAM" (Ha, Yeon, Yu):

* ``knn``          k-nearest neighbours; the covariance of a point is the
                   covariance of its k nearest neighbours (Sec. 3, definition
                   of the Gaussian set G = {X, C}).
* ``covariance``   that covariance, its decomposition C = R Lambda^2 R^T and
                   the plane / ellipse scale regularisations (Sec. 3.1.1,
                   Scale Regularization).
* ``se3``          the SE(3) exponential used for the pose update, and the
                   rotation logarithm used for error metrics.
* ``gicp``         the maximum-likelihood objective of Eq. (MLE_for_T),
                   minimised by Gauss-Newton with nearest-neighbour
                   correspondences recomputed every iteration (Sec. 3).

Every function is written for a reader to check against the paper by eye:
no blocking, fusion or reordering beyond what the definition states.
"""
from . import knn, covariance, se3, gicp

__all__ = ["knn", "covariance", "se3", "gicp"]
