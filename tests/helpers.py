"""Shared test helpers: map the library's slot-major ELL edge arrays onto the
oracle's CSR entries, and relative-error measures."""
import numpy as np


def ell_to_csr_index(col_ell, row_ptr, col_csr):
    """For each valid ELL entry (k, i) with j = col_ell[k, i] >= 0 return
    (mask, csr_index) so that csr arrays indexed by csr_index line up with
    ell_array[mask]."""
    W, N = col_ell.shape
    rows = np.broadcast_to(np.arange(N), (W, N))
    mask = col_ell >= 0
    key_ell = rows[mask].astype(np.int64) * N + col_ell[mask].astype(np.int64)
    row_csr = np.repeat(np.arange(N), np.diff(row_ptr)).astype(np.int64)
    key_csr = row_csr * N + col_csr
    order = np.argsort(key_csr)
    pos = np.searchsorted(key_csr[order], key_ell)
    assert np.array_equal(key_csr[order][pos], key_ell), "ELL and CSR patterns differ"
    return mask, order[pos]


def rel_err(a, b, axis=None):
    """max |a - b| / max |b| (per leading component when axis is given)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if axis is None:
        s = np.abs(b).max()
        return np.abs(a - b).max() / (s if s > 0 else 1.0)
    num = np.abs(a - b).max(axis=axis)
    den = np.abs(b).max(axis=axis)
    return num / np.where(den > 0, den, 1.0)


def state_scale(b):
    """Per-component max norm of an (nc, N) state; the momentum components
    share one scale (the largest of them)."""
    b = np.asarray(b)
    dim = b.shape[0] - 2
    scale = np.abs(b).max(axis=1)
    scale[1:1 + dim] = scale[1:1 + dim].max()
    return np.where(scale > 0, scale, 1.0)


def state_rel_err(a, b, scale=None):
    """Per-component relative max-norm error of two (nc, N) states, divided
    by state_scale(b), or by `scale` (e.g. the norm of the whole field when
    a and b are a sample of it)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if scale is None:
        scale = state_scale(b)
    return np.abs(a - b).max(axis=1) / scale
