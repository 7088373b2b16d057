"""CPU oracle of the iterative piecewise-planar stereo method (Pillai, Ramalingam and
Leonard, "High-Performance and Tunable Stereo Reconstruction", ICRA 2016).

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference the GPU path is
checked against. Only the tests, the package's smoke check and the CPU-baseline leg
of the benchmark may import it; the product path never calls it and it never calls
the product path. It shares no code, header, table or helper with the HIP library.

It restates the paper step by step in NumPy / Python integers:

* ``census``    census words and the high-gradient set (cost-evaluation section;
                high-gradient subset of Sec. III);
* ``matching``  support candidates and epipolar matching with a left-right check
                (Sec. III-A, "SparseStereo" / "SparseEpipolarStereo" of Alg. 1 / Alg. 4);
* ``fast``      FAST keypoints sampled from spatial bins, the paper's own support
                detector (Sec. III-A), as an alternative to the candidate grid;
* ``delaunay``  Delaunay triangulation of the supports (Sec. III-A), exact integer
                predicates with symbolic perturbation for ties;
* ``interp``    per-triangle disparity planes (Eq. 3) and the pixel-to-triangle
                lookup / interpolation (Sec. III-B, "DisparityInterpolation");
* ``refine``    CostEvaluation (Alg. 2) and DisparityRefinement (Alg. 3);
* ``resample``  SupportResampling (Alg. 4);
* ``solve``     Iterative Stereo Reconstruction (Alg. 1).

Where the paper is silent the oracle follows the readings listed in the design
document (census bit order, gradient operator, matcher acceptance rules, tie
breaking, rounding of a real disparity to a column, cell indexing).

Parity status: every function is pinned by the CPU tests (brute force, closed
forms, invariants, hand-derived cases); none is "parity unpinned". The end-to-end
multi-plane scenes are additionally compared only against this oracle (their
accuracy against the synthetic ground truth is context, not a pin).
"""
from .params import Params
from .census import census, high_gradient
from .matching import grid_candidates, match_point, sparse_stereo, hamming
from .fast import CIRCLE, fast_score, keypoints, fast_candidates
from .delaunay import triangulate, orient, incircle, incircle_sos
from .interp import plane_of, planes, interpolate
from .refine import cost_evaluation, disparity_refinement, Cell
from .resample import support_resampling
from .solve import solve, occupancy_size

__all__ = [
    "Params", "census", "high_gradient", "grid_candidates", "match_point", "sparse_stereo",
    "hamming", "triangulate", "orient", "incircle", "incircle_sos", "plane_of", "planes",
    "interpolate", "cost_evaluation", "disparity_refinement", "Cell", "support_resampling",
    "solve", "occupancy_size",
]
