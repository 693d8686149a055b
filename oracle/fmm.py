"""Reference 2-D Helmholtz FMM in plain numpy FP64 (test infrastructure).

Follows Sec. 5.1.1 (hierarchical quad-tree subdivision down to the leaf
level) and Sec. 5.1.2 (the calculation flow P2M -> M2M -> M2L -> L2L -> L2P,
plus P2P for the near field).  The paper gives no expansion formulas for 2-D
Helmholtz; this oracle uses the partial-wave expansions that follow from
Graf's addition theorem for cylinder functions (DLMF 10.23.7), written with

    in_v(z)  = J_v(k|z|)     exp(i v arg z)
    out_v(z) = H_v^(1)(k|z|) exp(i v arg z)

so that, for |b| < |a|,   out_n(a + b) = sum_m out_{n-m}(a) in_m(b)   and, for
all a, b,   in_n(a + b) = sum_m in_{n-m}(a) in_m(b).  From these:

    P2M  M_n  = sum_j q_j J_n(k rho_j) exp(-i n phi_j)   (rho, phi of y_j - c)
         far field  phi(x) = (i/4) sum_n M_n out_n(x - c)
    M2M  (c1 -> c2)  M'_l = sum_n M_n in_{n-l}(c2 - c1)
    M2L  (multipole at c -> local at c')  L_m = sum_n M_n out_{n-m}(c' - c)
    L2L  (c' -> c'') L''_l = sum_m L_m in_{m-l}(c'' - c')
    L2P  phi(x) = (i/4) sum_m L_m in_m(x - c')

Readings of points the paper leaves open:
* Tree: uniform depth L = max(2, ceil(log4(N / leaf))) over a square root box
  (smallest L with leaf * 4**L >= N); leaf <= 0 means one leaf (all pairs).
* Order per level: p_l = p + floor(k d_l / 2), d_l the box diagonal; the index
  range is n = -p_l..p_l (2 p_l + 1 coefficients).
* Well-separated means "not adjacent": the interaction list of a box is the
  children of its parent's neighbours that are not its own neighbours.
* P2P runs over the 3 x 3 neighbouring leaves; zero-distance pairs add nothing.
"""

import math

import numpy as np
from scipy.special import hankel1, jv

from .kernel import dgreen_dn, green


def tree_depth(n_points, leaf):
    """Uniform depth: 0 for leaf <= 0 (one leaf), else max(2, ceil(log4(N/leaf)))."""
    if leaf <= 0:
        return 0
    L = 0
    while leaf * (4 ** L) < n_points:
        L += 1
    return max(2, L)


def level_orders(k, p, L, side):
    """p_l = p + floor(k d_l / 2) with d_l = sqrt(2) * side / 2**l."""
    return [p + int(math.floor(k * math.sqrt(2.0) * side / 2 ** l / 2.0)) for l in range(L + 1)]


def _in(nu, z, k):
    return jv(nu, k * np.abs(z)) * np.exp(1j * nu * np.angle(z))


def _out(nu, z, k):
    return hankel1(nu, k * np.abs(z)) * np.exp(1j * nu * np.angle(z))


def leaf_coords(xy, L, root):
    x0, y0, side = root
    nb = 2 ** L
    ix = np.clip(np.floor((xy[:, 0] - x0) / side * nb).astype(np.int64), 0, nb - 1)
    iy = np.clip(np.floor((xy[:, 1] - y0) / side * nb).astype(np.int64), 0, nb - 1)
    return ix, iy


def box_center(l, bx, by, root):
    x0, y0, side = root
    s = side / 2 ** l
    return (x0 + (bx + 0.5) * s) + 1j * (y0 + (by + 0.5) * s)


def fmm(xy, q, k, p, leaf, root=(0.0, 0.0, 1.0), targets=None, return_stages=False, normals=None):
    """Reference FMM: phi_i ~ sum_{j != i} q_j (i/4) H0(k |x_i - x_j|).

    xy : (N, 2) float64 points (sources = targets).  q : (N,) or (N, nrhs).
    targets : optional integer indices; only those potentials are computed
              (the downward pass runs only on their ancestors).
    normals : optional (N, 2) unit normals; the sources are then dipoles and
              the sum is phi_i ~ sum_j q_j dG/dn_j(x_i, x_j) (the double layer
              of Sec. 5.2).  Only P2M and P2P change: the multipole of a
              dipole is the derivative of the monopole's along n at the source,
                  M_n = q (n . grad_y) [J_n(k rho) e^{-i n phi}]
                      = q (k/2) [conj(nu) b_{n-1} - nu b_{n+1}],
              b_m = J_m(k rho) e^{-i m phi}, nu = n_x + i n_y, which follows
              from the ladder relations (d/dx +- i d/dy) of the cylinder
              functions (DLMF 10.6.2).
    Returns phi for the targets (all points by default) and, if asked, a dict
    with the per-level orders and the multipole/local arrays.
    """
    xy = np.asarray(xy, dtype=np.float64)
    q = np.asarray(q, dtype=np.complex128)
    if normals is not None:
        normals = np.asarray(normals, dtype=np.float64)
    squeeze = q.ndim == 1
    if squeeze:
        q = q[:, None]
    N, nrhs = q.shape
    tidx = np.arange(N) if targets is None else np.asarray(targets, dtype=np.int64)
    x0, y0, side = root
    L = tree_depth(N, leaf)
    ix, iy = leaf_coords(xy, L, root)
    pts = xy[:, 0] + 1j * xy[:, 1]
    pl = level_orders(k, p, L, side)
    stages = {"L": L, "orders": pl, "M": {}, "Lc": {}}

    phi = np.zeros((tidx.size, nrhs), dtype=np.complex128)

    if L >= 2:
        # ---- P2M at the leaves
        P = pl[L]
        n = np.arange(-P, P + 1)
        c = box_center(L, ix, iy, root)
        rel = pts - c
        def b(m):
            return jv(m[None, :], k * np.abs(rel)[:, None]) * np.exp(-1j * m[None, :] * np.angle(rel)[:, None])

        if normals is None:
            terms = b(n)
        else:
            nu = (normals[:, 0] + 1j * normals[:, 1])[:, None]
            terms = 0.5 * k * (np.conj(nu) * b(n - 1) - nu * b(n + 1))
        M = {L: np.zeros((2 ** L, 2 ** L, 2 * P + 1, nrhs), dtype=np.complex128)}
        np.add.at(M[L], (ix, iy), terms[:, :, None] * q[:, None, :])

        # ---- M2M, levels L-1 .. 2
        for l in range(L - 1, 1, -1):
            Pp, Pc = pl[l], pl[l + 1]
            nbp = 2 ** l
            M[l] = np.zeros((nbp, nbp, 2 * Pp + 1, nrhs), dtype=np.complex128)
            sc = side / 2 ** (l + 1)
            lp = np.arange(-Pp, Pp + 1)[:, None]
            nc = np.arange(-Pc, Pc + 1)[None, :]
            for cx in (0, 1):
                for cy in (0, 1):
                    # child centre minus parent centre
                    dch = (cx - 0.5) * sc + 1j * (cy - 0.5) * sc
                    W = _in(nc - lp, -dch, k)  # in_{n-l}(c_parent - c_child)
                    child = M[l + 1][cx::2, cy::2]
                    M[l] += np.einsum("ln,xynr->xylr", W, child)

        # ---- which boxes need local expansions (ancestors of target leaves)
        need = {L: np.zeros((2 ** L, 2 ** L), dtype=bool)}
        need[L][ix[tidx], iy[tidx]] = True
        for l in range(L - 1, 1, -1):
            nb = 2 ** l
            need[l] = need[l + 1].reshape(nb, 2, nb, 2).any(axis=(1, 3))

        # ---- M2L at every level 2..L over the interaction lists
        Lc = {}
        for l in range(2, L + 1):
            Pl = pl[l]
            nb = 2 ** l
            s = side / 2 ** l
            Lc[l] = np.zeros((nb, nb, 2 * Pl + 1, nrhs), dtype=np.complex128)
            mm = np.arange(-Pl, Pl + 1)[:, None]
            nn = np.arange(-Pl, Pl + 1)[None, :]
            bx, by = np.nonzero(need[l])
            for ox in range(-3, 4):
                for oy in range(-3, 4):
                    if max(abs(ox), abs(oy)) < 2:
                        continue
                    sx, sy = bx + ox, by + oy
                    ok = (sx >= 0) & (sx < nb) & (sy >= 0) & (sy < nb)
                    ok &= (np.abs(np.floor_divide(sx, 2) - bx // 2) <= 1)
                    ok &= (np.abs(np.floor_divide(sy, 2) - by // 2) <= 1)
                    if not ok.any():
                        continue
                    # c_target - c_source = -(ox, oy) * s
                    T = _out(nn - mm, -(ox + 1j * oy) * s, k)
                    Lc[l][bx[ok], by[ok]] += np.einsum("mn,bnr->bmr", T, M[l][sx[ok], sy[ok]])

        # ---- L2L, levels 2 .. L-1
        for l in range(2, L):
            Pp, Pc = pl[l], pl[l + 1]
            sc = side / 2 ** (l + 1)
            lc = np.arange(-Pc, Pc + 1)[:, None]
            mp_ = np.arange(-Pp, Pp + 1)[None, :]
            for cx in (0, 1):
                for cy in (0, 1):
                    dch = (cx - 0.5) * sc + 1j * (cy - 0.5) * sc
                    W = _in(mp_ - lc, dch, k)  # in_{m-l}(c_child - c_parent)
                    Lc[l + 1][cx::2, cy::2] += np.einsum("lm,xymr->xylr", W, Lc[l])

        # ---- L2P at the targets
        P = pl[L]
        n = np.arange(-P, P + 1)
        ct = box_center(L, ix[tidx], iy[tidx], root)
        rel = pts[tidx] - ct
        basis = jv(n[None, :], k * np.abs(rel)[:, None]) * np.exp(1j * n[None, :] * np.angle(rel)[:, None])
        phi += 0.25j * np.einsum("tn,tnr->tr", basis, Lc[L][ix[tidx], iy[tidx]])
        stages["M"], stages["Lc"] = M, Lc

    # ---- P2P over the 3 x 3 neighbouring leaves (with L < 2 every leaf is
    #      adjacent to every other, so this is the all-pairs sum)
    nbL = 2 ** L
    key = ix * nbL + iy
    order = np.argsort(key, kind="stable")
    starts = np.searchsorted(key[order], np.arange(nbL * nbL + 1))
    tkey = key[tidx]
    for tk in np.unique(tkey):
        rows = np.nonzero(tkey == tk)[0]
        bx, by = divmod(int(tk), nbL)
        src = []
        for sx in range(max(bx - 1, 0), min(bx + 2, nbL)):
            for sy in range(max(by - 1, 0), min(by + 2, nbL)):
                sk = sx * nbL + sy
                src.append(order[starts[sk]:starts[sk + 1]])
        src = np.concatenate(src)
        r = np.abs(pts[tidx[rows]][:, None] - pts[src][None, :])
        g = np.zeros(r.shape, dtype=np.complex128)
        use = r > 0
        if normals is None:
            g[use] = green(r[use], k)
        else:
            X = np.broadcast_to(xy[tidx[rows]][:, None, :], r.shape + (2,))
            Y = np.broadcast_to(xy[src][None, :, :], r.shape + (2,))
            Nn = np.broadcast_to(normals[src][None, :, :], r.shape + (2,))
            g[use] = dgreen_dn(X[use], Y[use], Nn[use], k)
        phi[rows] += g @ q[src]

    phi = phi[:, 0] if squeeze else phi
    return (phi, stages) if return_stages else phi
