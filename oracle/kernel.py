"""The 2-D Helmholtz kernel and the direct N-body sum (test infrastructure).

Follows:
* Sec. 5.2, 2-D free-space Green's function: G(P,Q) = (i/4) H0^(1)(k r),
  r = |P - Q|.  H0^(1) is taken from ``scipy.special.hankel1`` (a library
  primitive).
* Sec. 5.1, the N-body sum f(y_j) = sum_i w_i K(y_j, x_i).

* Sec. 5.2, the normal derivative of the 2-D Green's function at the source
  point: dG/dn(P, Q) = -(i k / 4) H1^(1)(k r) r_n with r_n the derivative of
  r = |P - Q| along the unit normal n at Q, r_n = (Q - P).n / r; written here
  as (i k / 4) H1(k r) (P - Q).n / r.  H1^(1) from ``scipy.special.hankel1``.

Reading (paper silent): pairs at distance exactly zero (a point with itself,
or two coincident distinct points) contribute nothing, for G and for dG/dn.
"""

import os

import numpy as np
from scipy.special import hankel1


def green(r, k):
    """G = (i/4) H0^(1)(k r) for r > 0 (Sec. 5.2, 2-D Green's function)."""
    return 0.25j * hankel1(0, k * np.asarray(r, dtype=np.float64))


def dgreen_dn(x, y, normal, k):
    """dG/dn_y (x, y) = (i k / 4) H1(k r) (x - y).n / r for r > 0 (Sec. 5.2, 2-D kernel).

    x, y : (..., 2) points; normal : (..., 2) unit normals at y.
    """
    x, y, normal = (np.asarray(a, dtype=np.float64) for a in (x, y, normal))
    d = x - y
    r = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
    rn = (d[..., 0] * normal[..., 0] + d[..., 1] * normal[..., 1]) / r
    return 0.25j * k * hankel1(1, k * r) * rn


def direct_sum_dipole(src, q, normals, k, tgt=None, chunk=None):
    """phi[i, c] = sum_{j : |t_i - s_j| > 0} q[j, c] dG/dn_j(t_i, s_j): the double-layer sum."""
    src = np.asarray(src, dtype=np.float64)
    normals = np.asarray(normals, dtype=np.float64)
    q = np.asarray(q, dtype=np.complex128)
    squeeze = q.ndim == 1
    if squeeze:
        q = q[:, None]
    tgt = src if tgt is None else np.asarray(tgt, dtype=np.float64)
    if chunk is None:
        chunk = max(1, min(256, (1 << 22) // max(1, src.shape[0])))
    out = np.zeros((tgt.shape[0], q.shape[1]), dtype=np.complex128)
    for a in range(0, tgt.shape[0], chunk):
        t = tgt[a:a + chunk]
        d = t[:, None, :] - src[None, :, :]
        r = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
        g = np.zeros(r.shape, dtype=np.complex128)
        nz = r > 0
        nrm = np.broadcast_to(normals[None, :, :], d.shape)
        g[nz] = dgreen_dn(np.broadcast_to(t[:, None, :], d.shape)[nz], np.broadcast_to(src[None], d.shape)[nz],
                          nrm[nz], k)
        out[a:a + chunk] = g @ q
    return out[:, 0] if squeeze else out


def direct_sum(src, q, k, tgt=None, chunk=None):
    """phi[i, c] = sum_{j : |t_i - s_j| > 0} q[j, c] G(t_i, s_j)   (Sec. 5.1 N-body sum).

    src : (N, 2) float64 source positions.
    q   : (N,) or (N, nrhs) complex weights.
    tgt : (M, 2) target positions; defaults to the sources themselves.
    Returns (M,) or (M, nrhs) complex128.
    """
    src = np.asarray(src, dtype=np.float64)
    q = np.asarray(q, dtype=np.complex128)
    squeeze = q.ndim == 1
    if squeeze:
        q = q[:, None]
    tgt = src if tgt is None else np.asarray(tgt, dtype=np.float64)
    if chunk is None:  # bound the (targets x sources) work arrays to ~2^22 entries
        chunk = max(1, min(256, (1 << 22) // max(1, src.shape[0])))
    out = np.zeros((tgt.shape[0], q.shape[1]), dtype=np.complex128)
    for a in range(0, tgt.shape[0], chunk):
        t = tgt[a:a + chunk]
        d = t[:, None, :] - src[None, :, :]
        r = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
        g = np.zeros(r.shape, dtype=np.complex128)
        nz = r > 0
        g[nz] = green(r[nz], k)
        out[a:a + chunk] = g @ q
    return out[:, 0] if squeeze else out


def _direct_sum_rows(args):
    src, q, k, tgt = args
    return direct_sum(src, q, k, tgt=tgt)


def direct_sum_parallel(src, q, k, tgt, workers=None):
    """The same sum as ``direct_sum``, split over target chunks in a process pool.

    Used only to time the oracle and to check sampled targets of large runs.
    """
    import multiprocessing as mp

    workers = workers or len(os.sched_getaffinity(0))
    tgt = np.asarray(tgt, dtype=np.float64)
    parts = np.array_split(np.arange(tgt.shape[0]), max(1, workers))
    parts = [p for p in parts if p.size]
    if len(parts) == 1:
        return direct_sum(src, q, k, tgt=tgt)
    ctx = mp.get_context("fork")
    with ctx.Pool(len(parts)) as pool:
        res = pool.map(_direct_sum_rows, [(src, q, k, tgt[p]) for p in parts])
    return np.concatenate(res, axis=0)
