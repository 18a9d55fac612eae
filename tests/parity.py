"""Comparison helpers of the GPU parity tests (test infrastructure only).

Two measures of the difference between a GPU result a and the oracle's b,
both interleaved [n_nodes, 2] (field 0 = phi rows, field 1 = u rows):

* rel(a, b): norm-wise, |a - b|_2 / |b|_2;
* field_maxabs(a, b): per field, the largest elementwise difference over the
  largest reference entry of that field, max_i |a_if - b_if| / max_i |b_if|,
  so that a wrong entry in a small field (or a few wrong nodes in a large
  vector) is not averaged away by the other field or the rest of the nodes.

Newton solutions are compared on their increments U - U_start: the bulk values
+-1 of a phase field would otherwise dominate both measures.
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def field_maxabs(a, b):
    a = np.asarray(a, dtype=float).reshape(-1, 2)
    b = np.asarray(b, dtype=float).reshape(-1, 2)
    out = []
    whole = float(np.abs(b).max()) if b.size else 0.0
    for f in range(2):
        scale = float(np.abs(b[:, f]).max()) if b.size else 0.0
        if scale == 0.0:
            scale = whole if whole > 0.0 else 1.0
        out.append(float(np.abs(a[:, f] - b[:, f]).max()) / scale if b.size else 0.0)
    return out


def check(a, b, tol, what="", field_tol=None):
    """Assert rel(a, b) <= tol and every field_maxabs(a, b) <= field_tol (default tol)."""
    r = rel(a, b)
    m = field_maxabs(a, b)
    ft = tol if field_tol is None else field_tol
    print(f"[parity] {what}: rel {r:.3e}, per-field max-abs phi {m[0]:.3e} u {m[1]:.3e} "
          f"(tol {tol:.0e}, field tol {ft:.0e})", flush=True)
    assert r <= tol, (what, r, m)
    assert max(m) <= ft, (what, r, m)
    return r, m


def check_increment(a, b, start, tol, what="", field_tol=None):
    """check() on a - start against b - start (Newton increments)."""
    s = np.asarray(start, dtype=float).reshape(-1, 2)
    return check(np.asarray(a).reshape(-1, 2) - s, np.asarray(b).reshape(-1, 2) - s, tol,
                 what + " (increment)", field_tol)
