"""Error measures of the GPU parity tests: a global relative l2 error over the packed vector and,
per (field, m) block of the packed layout, the largest element error relative to the largest
element of that block (so that small fields and high-degree tails are judged on their own
scale, not hidden in a global norm)."""
import numpy as np

FIELDS = ("e", "f", "T")

# Per-block bar of the FP64 path (every (field, m) block to 1e-11 of its own largest element).
FP64_BLOCK = 1e-11


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def block_errors(lay, y, ref):
    """{(field, m): max |y - ref| / max |ref|} over the (field, m) blocks of the packed layout.
    A block whose reference is identically zero is judged absolutely (max |y|)."""
    out = {}
    for fld in range(3):
        for k, m in enumerate(lay.ms):
            o = lay.offset(fld, k, m)
            n = 2 * lay.N * lay.nl[k]
            r = ref[o:o + n]
            d = np.abs(y[o:o + n] - r).max()
            s = np.abs(r).max()
            out[(FIELDS[fld], m)] = float(d / s) if s > 0 else float(d)
    return out


def check(lay, y, ref, tol, block_tol=None, label=""):
    """Assert the global relative error <= tol and every block error <= block_tol (default tol);
    returns (global error, worst block, its error)."""
    g = rel(y, ref)
    be = block_errors(lay, y, ref)
    worst = max(be, key=be.get)
    print(f"{label} rel err {g:.2e}; worst (field, m) block {worst} {be[worst]:.2e}", flush=True)
    assert g <= tol, (label, g)
    bt = tol if block_tol is None else block_tol
    assert be[worst] <= bt, (label, worst, be[worst])
    return g, worst, be[worst]
