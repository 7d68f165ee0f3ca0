"""Parity bars shared by the GPU tests (helpers only; nothing collected here)."""
import numpy as np

U = np.finfo(np.float64).eps / 2      # unit roundoff


def history_bound(Jo, hier_levels, h_o, blocks=("pp", "S")):
    """Per-iteration bound on |history_gpu - history_oracle| (the relative
    residual estimates of the first ten iterations).

    Multi-level hierarchies: the two V-cycles agree to ~1e-15 relative
    (identical setups; only row sums and the small coarsest solve differ in
    rounding order), and the estimates agree to 1e-8 relative, iteration by
    iteration.

    A one-level hierarchy is the dense coarse solve of the whole block: the
    GPU applies a Gauss-Jordan inverse, the oracle LU solves.  Both are
    backward stable, so their outputs differ by up to u kappa(A) relative,
    u the unit roundoff and kappa the block's 2-norm condition number; the
    minimal residual over the Krylov space is Lipschitz in the operator, so
    the estimates differ by at most about u kappa ||b|| = u kappa h_0 (for
    the W1 pressure block kappa = 2e6, for W2g 5e7: u kappa h_0 = 2e-10 and
    5e-9 h_0, measured 6e-13 and 2e-11 h_0).  Where that is looser than the
    relative bar (late iterations of a one-level solve, estimates near
    1e-10 h_0) it is the one tested."""
    rel = 1e-8 * np.asarray(h_o)
    if min(hier_levels) > 1:
        return rel
    kappa = max(np.linalg.cond(Jo.block(k).toarray()) for k in blocks)
    return np.maximum(rel, U * kappa * h_o[0])
