"""ORACLE — TEST INFRASTRUCTURE ONLY.

Plain-loop definition of the masked semiring matrix-vector products
mxv and vxm (Section 3.3 and the mxv figure caption: w = A u .* mask over a
semiring; vxm is mxv with A transposed, per the caption of the operation
decomposition figure).  Pure Python over dictionaries, meant for small
inputs only.  Only tests/, the smoke check and the benchmark's CPU-baseline
leg may use it.

Conventions (the paper's masking semantics, Section 3.2.1, plus the
GraphBLAS C API for accum and REPLACE, which the paper's text defers to):

* A is a list of (i, j, a) triples (a = 1 for a structure-only matrix),
  at most one triple per (i, j).
* Vectors are dicts index -> value; absent index = no entry.
* mxv:  t(i) = (+)_{j : A(i,j) and u(j) present} A(i,j) (x) u(j)
  vxm:  t(j) = (+)_{i : A(i,j) and u(i) present} u(i) (x) A(i,j)
  t(i) exists iff its index set is non-empty.
* m(i) = i present in mask and mask(i) != 0 (value mask), or i present
  (structural mask); allowed(i) = (no mask) or (m(i) xor complement).
* z = t with no accum; with accum, z(i) = accum(w_old(i), t(i)) where both
  exist, else whichever exists.
* w_new(i) = z(i) (or absent) where allowed(i); elsewhere w_old(i), or
  absent under REPLACE.
"""
from __future__ import annotations

import math

INT32_MAX = 2**31 - 1

# semiring name -> (add, mul, identity, cast)
def _lor(x, y):
    return bool(x) or bool(y)


def _land(x, y):
    return bool(x) and bool(y)


SEMIRINGS = {
    "lor_land": (_lor, _land, False, bool),
    "min_plus": (min, lambda x, y: x + y, math.inf, float),
    "plus_times": (lambda x, y: x + y, lambda x, y: x * y, 0.0, float),
    "min_first": (min, lambda x, y: x, INT32_MAX, int),
    "min_second": (min, lambda x, y: y, INT32_MAX, int),
}

ACCUMS = {
    None: None,
    "min": min,
    "plus": lambda x, y: x + y,
    "lor": _lor,
}


def _mask_allowed(i, mask, complement, structural):
    if mask is None:
        return True
    if structural:
        m = i in mask
    else:
        m = i in mask and mask[i] != 0
    return m != complement


def mxv(n_out, A, u, *, semiring, w_old=None, mask=None, complement=False,
        structural=False, accum=None, replace=False, transpose=False):
    """w = A' u .* mask over `semiring` (A' = A, or A^T when transpose)."""
    add, mul, _ident, cast = SEMIRINGS[semiring]
    w_old = {} if w_old is None else w_old
    t = {}
    for (i, j, a) in A:
        if transpose:
            i, j = j, i
        if j in u:
            prod = mul(cast(a), cast(u[j]))
            t[i] = add(t[i], prod) if i in t else prod
    return _apply(n_out, t, w_old, mask, complement, structural, accum, replace)


def vxm(n_out, A, u, *, semiring, w_old=None, mask=None, complement=False,
        structural=False, accum=None, replace=False, transpose=False):
    """w = u A' .* mask: t(j) = (+)_i u(i) (x) A'(i, j)."""
    add, mul, _ident, cast = SEMIRINGS[semiring]
    w_old = {} if w_old is None else w_old
    t = {}
    for (i, j, a) in A:
        if transpose:
            i, j = j, i
        if i in u:
            prod = mul(cast(u[i]), cast(a))
            t[j] = add(t[j], prod) if j in t else prod
    return _apply(n_out, t, w_old, mask, complement, structural, accum, replace)


def _apply(n_out, t, w_old, mask, complement, structural, accum, replace):
    acc = ACCUMS[accum]
    if acc is None:
        z = dict(t)
    else:
        z = {}
        for i in set(t) | set(w_old):
            if i in t and i in w_old:
                z[i] = acc(w_old[i], t[i])
            elif i in t:
                z[i] = t[i]
            else:
                z[i] = w_old[i]
    w = {}
    for i in range(n_out):
        if _mask_allowed(i, mask, complement, structural):
            if i in z:
                w[i] = z[i]
        elif not replace and i in w_old:
            w[i] = w_old[i]
    return w
