"""Parity bounds for the network kernels, shared by the GPU tests and by the
CPU test that shows they reject a wrong network.  Each check has two tiers.

Tier 1, every entry: the worst case the arithmetic allows.
  Forward.  The kernel accumulates binary16 products in binary32 where the
  oracle uses binary64, so a hidden activation rounded to binary16 may land
  one unit in the last place (at most 2^-10 of its value) away.  There are
  two such rounding points; what reaches the output through active units is
  bounded by the oracle's magnitude (|w| times the previous layer's
  magnitude over active units), so |gpu - oracle| <= 2 * 2^-10 * mag.
  Backward, against the oracle's bfloat16 mode (which rounds the same
  operands): a masked hidden gradient rounded to bfloat16 may land one unit
  (at most 2^-7 of its value) away, and a flipped binary16 activation may
  round to a neighbouring bfloat16 operand; both travel through at most two
  more products, so 2^-5 of the magnitude covers them.
Tier 2, the distribution: a rounding flip moves an output by one unit of
  one activation's share of the sum, far below 2^-14 of the magnitude; so
  at most 0.1 % of the entries (and at least one allowed) may differ by more
  than 2^-14 of the magnitude.  A dropped hidden unit or a transposed weight
  moves a large share of the entries by much more (tests/test_tolerances.py).
"""
import numpy as np

TINY = 2.0 ** -24          # smallest binary16 subnormal: the absolute floor
FWD_BOUND = 2.0 ** -9
BWD_BOUND = 2.0 ** -5
TYPICAL = 2.0 ** -14
TYPICAL_SHARE = 1e-3


def _check(name, got, ref, mag, bound):
    err = np.abs(np.asarray(got, np.float64) - ref)
    tol = bound * mag + TINY
    if not (err <= tol).all():
        i = np.unravel_index(np.argmax(err / tol), err.shape)
        return f"{name}: entry {i} err {err[i]:.3e} > bound {tol[i]:.3e}"
    wide = int(np.count_nonzero(err > TYPICAL * mag + TINY))
    allowed = max(1, int(TYPICAL_SHARE * err.size))
    if wide > allowed:
        return f"{name}: {wide} of {err.size} entries beyond 2^-14 of the magnitude (at most {allowed})"
    return None


def mlp_fwd_problem(got, ref, mag):
    """None if the forward output `got` passes against the oracle's
    (ref, mag); otherwise a description of the first failure."""
    return _check("y", got, ref, mag, FWD_BOUND)


def mlp_bwd_problem(got, ref, keys=("d_x", "dW1", "dW2", "dW3")):
    """None if every backward result in `got` passes against the oracle's
    bfloat16-mode results `ref` (with magnitudes, mlp_bwd(..., with_mag=True))."""
    for k in keys:
        p = _check(k, got[k], ref[k], ref["mag_" + k], BWD_BOUND)
        if p:
            return p
    return None


# rounded operands on each backward result's path (operand roundings of at
# most 2^-8 each), for the error against the exact mode
BF16_OPERANDS = {"dW3": 2, "dW2": 4, "dW1": 6, "d_x": 6}


def mlp_bwd_vs_exact(got, exact):
    """Error of the bfloat16 backward against the network's exact
    derivative: per result, max and p99 of |err| / magnitude, and the bound
    (number of rounded operands on the path) * 2^-8 plus the tier-1 margin."""
    out = {}
    for k, r in BF16_OPERANDS.items():
        m = exact["mag_" + k]
        rel = np.abs(np.asarray(got[k], np.float64) - exact[k]) / np.maximum(m, 1e-300)
        bound = r * 2.0 ** -8 * 1.01 + BWD_BOUND
        out[k] = {"max": float(rel.max()), "p99": float(np.percentile(rel, 99)), "bound": bound,
                  "ok": bool((np.abs(np.asarray(got[k], np.float64) - exact[k]) <= bound * m + TINY).all())}
    return out
