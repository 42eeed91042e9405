"""Comparison of a GPU result with the oracle's, element by element.

The parity bar is a relative L2 error over the whole state (the error norm
of the paper's convergence studies), and, so that a wrong low-population
surface or a few wrong elements cannot hide inside that sum, also

  * per surface: ||got_s - ref_s|| <= tol * max(||ref_s||, floor * ||ref||),
    relative to the surface's own norm unless that is below `floor` of the
    total (an empty or nearly empty surface is held to tol * floor * ||ref||);
  * per element: max |got - ref| <= tol * max |ref|.
"""
import numpy as np


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def parity_errors(got, ref, floor=1e-2):
    """(whole-state relative L2, worst per-surface ratio, max-abs ratio); the
    leading axis of got/ref is the surface (a batch axis before it is
    flattened into it)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    tot = float(np.linalg.norm(ref.ravel()))
    whole = float(np.linalg.norm((got - ref).ravel())) / tot
    g = got.reshape(got.shape[0] if got.ndim > 1 else 1, -1)
    r = ref.reshape(g.shape)
    per = 0.0
    for s in range(g.shape[0]):
        den = max(float(np.linalg.norm(r[s])), floor * tot)
        per = max(per, float(np.linalg.norm(g[s] - r[s])) / den)
    mx = float(np.max(np.abs(got - ref))) / float(np.max(np.abs(ref)))
    return whole, per, mx


def assert_parity(got, ref, tol, what="", floor=1e-2, elem_tol=None):
    """Whole-state relative L2 below tol; per-surface and max-abs ratios
    below elem_tol (default tol; FP32 results, whose rounding errors are not
    spread evenly, state a larger one)."""
    elem_tol = tol if elem_tol is None else elem_tol
    whole, per, mx = parity_errors(got, ref, floor)
    print(f"[parity] {what} rel L2 {whole:.2e}, worst surface {per:.2e}, max-abs {mx:.2e}",
          flush=True)
    assert whole < tol, f"{what}: relative L2 {whole:.3e} >= {tol:.1e}"
    assert per < elem_tol, f"{what}: per-surface error {per:.3e} >= {elem_tol:.1e}"
    assert mx < elem_tol, f"{what}: max-abs error {mx:.3e} >= {elem_tol:.1e}"
    return whole, per, mx
