"""Reference 3-D Helmholtz FMM on an oct-tree, plain numpy FP64 (test
infrastructure only; nothing in the product imports it).

Sec. 5.1.1 describes the 3-D decomposition as an oct-tree, Sec. 5.1.2 the
calculation flow P2M -> M2M -> M2L -> L2L -> L2P with P2P for the near
field, and Sec. 5.2 the 3-D free-space kernel G(P, Q) = exp(i k r) / (4 pi r).
The paper gives no 3-D expansion formulas (its 3-D runs use a library); this
oracle uses the partial-wave expansions of the addition theorem of the
spherical Hankel function, written with

    R_n^m(x) = j_n(k|x|) Y_n^m(x/|x|)        (regular)
    S_n^m(x) = h_n(k|x|) Y_n^m(x/|x|)        (singular, h_n = j_n + i y_n)

Y_n^m orthonormal on the sphere with the Condon-Shortley phase (scipy's
sph_harm_y), n = 0..p, m = -n..n, coefficient index n^2 + n + m.

    G(x, y) = i k sum_{n,m} S_n^m(x - c) conj(R_n^m(y - c))   for |y-c| < |x-c|
    P2M  M_nm = i k sum_j q_j conj(R_n^m(y_j - c)); far field sum M_nm S_n^m(x - c)
    P2L  L_nm = i k q conj(Y_n^m(u)) h_n(k|y - c|),  u = (y - c)/|y - c|
    L2P  phi(x) = sum L_nm R_n^m(x - c)

Translations, from the plane-wave form of R_n^m and the product of two
spherical harmonics (Gaunt coefficients):

    (F)_{n'm', nm}(t) = 4 pi sum_l i^(n' + l - n) f_l(k|t|) conj(Y_l^(m'-m)(t/|t|))
                        * Gaunt(n', m'; l, m' - m; n, m)
    Gaunt(n', m'; l, mu; n, m) = integral of conj(Y_n'^m') Y_l^mu Y_n^m over the sphere

with f_l = j_l for the regular-to-regular form (R|R) and f_l = h_l for the
singular-to-regular form (S|R).  Then

    M2M  (child centre c -> parent centre c')  M'_{n'm'} = sum (R|R)(c' - c) M_nm
    M2L  (source box c_s -> target box c_t)    L_{n'm'}  = sum (S|R)(c_t - c_s) M_nm
    L2L  (parent c' -> child c'')              L''_{n'm'} = sum (R|R)(c'' - c') L_nm

Readings of points the paper leaves open (3-D):
* Tree: uniform depth L = max(2, smallest L with leaf * 8**L >= N) over a cube
  root box; leaf <= 0 means one leaf (all pairs).
* Order per level: p_l = p + floor(k d_l / 2), d_l = sqrt(3) side / 2**l (box
  diameter), as in the 2-D reading with the 3-D diameter.
* Well-separated means "not adjacent": the interaction list of a box is the
  children of its parent's 27 neighbours that are not its own neighbours
  (189 boxes inside the domain).
* P2P runs over the 27 neighbouring leaves (the leaf itself included);
  zero-distance pairs add nothing.
"""

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np
from scipy.special import spherical_jn, spherical_yn, sph_harm_y


# ------------------------------------------------------------------ kernel
def green3(r, k):
    """G = exp(i k r) / (4 pi r) (Sec. 5.2, 3-D Green's function)."""
    r = np.asarray(r, dtype=np.float64)
    return np.exp(1j * k * r) / (4.0 * math.pi * r)


def direct_sum3(xyz, q, k, targets=None, chunk=256):
    """phi_i = sum_{j, r_ij != 0} G(|x_i - y_j|) q_j (the N-body sum of Sec. 5.1
    with the 3-D kernel).  Targets default to the sources; zero-distance pairs
    add nothing.  Chunked over targets only (no reordering of the sum)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    q = np.asarray(q, dtype=np.complex128)
    tgt = xyz if targets is None else np.asarray(targets, dtype=np.float64)
    out = np.zeros(len(tgt), dtype=np.complex128)
    for a in range(0, len(tgt), chunk):
        d = tgt[a:a + chunk, None, :] - xyz[None, :, :]
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.where(r > 0, np.exp(1j * k * r) / (4.0 * math.pi * np.where(r > 0, r, 1.0)), 0.0)
        out[a:a + chunk] = g @ q
    return out


# ------------------------------------------------------------------ tree
def tree_depth3(n_points, leaf):
    """0 for leaf <= 0 (one leaf), else max(2, smallest L with leaf * 8**L >= N)."""
    if leaf <= 0:
        return 0
    L = 0
    while leaf * (8 ** L) < n_points:
        L += 1
    return max(2, L)


def level_orders3(k, p, L, side=1.0):
    """p_l = p + floor(k d_l / 2), d_l = sqrt(3) side / 2**l."""
    return [p + int(math.floor(k * math.sqrt(3.0) * side / 2 ** l / 2.0)) for l in range(L + 1)]


def interaction_offsets(parity):
    """Offsets d = target - source (in boxes of the level) of the interaction
    list of a box whose index has the given parity (px, py, pz): sources are
    children of the parent's neighbours, so d_x runs over [p_x - 3, p_x + 2],
    and neighbours (max |d| <= 1) are excluded: 189 offsets."""
    rng = [range(p - 3, p + 3) for p in parity]
    return [(dx, dy, dz) for dx in rng[0] for dy in rng[1] for dz in rng[2]
            if max(abs(dx), abs(dy), abs(dz)) >= 2]


# ------------------------------------------------------------------ special functions
def _cidx(n, m):
    return n * n + n + m


def _sph(xyz):
    """|x|, polar angle, azimuth of each row."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    r = np.sqrt(x * x + y * y + z * z)
    theta = np.arccos(np.clip(np.where(r > 0, z / np.where(r > 0, r, 1.0), 1.0), -1.0, 1.0))
    phi = np.arctan2(y, x)
    return r, theta, phi


def _Y(p, theta, phi):
    """Y_n^m(theta, phi) for n <= p, all m; shape (..., (p+1)^2)."""
    out = np.zeros(np.shape(theta) + ((p + 1) ** 2,), dtype=np.complex128)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            out[..., _cidx(n, m)] = sph_harm_y(n, m, theta, phi)
    return out


def _radial(p, x, kind):
    """j_n(x) ('j') or h_n(x) = j_n + i y_n ('h') for n <= p, broadcast to the
    coefficient layout (each n repeated 2n+1 times)."""
    x = np.asarray(x, dtype=np.float64)
    cols = []
    for n in range(p + 1):
        v = spherical_jn(n, x).astype(np.complex128)
        if kind == "h":
            v = v + 1j * spherical_yn(n, x)
        cols.extend([v] * (2 * n + 1))
    return np.stack(cols, axis=-1)


def basis_R(p, d, k):
    """R_n^m(d) for rows d; shape (N, (p+1)^2)."""
    r, th, ph = _sph(np.asarray(d, dtype=np.float64))
    return _radial(p, k * r, "j") * _Y(p, th, ph)


def basis_S(p, d, k):
    """S_n^m(d) for rows d (all nonzero); shape (N, (p+1)^2)."""
    r, th, ph = _sph(np.asarray(d, dtype=np.float64))
    return _radial(p, k * r, "h") * _Y(p, th, ph)


# ------------------------------------------------------------------ Gaunt coefficients
@lru_cache(maxsize=None)
def wigner3j(j1, j2, j3, m1, m2, m3):
    """Wigner 3j symbol by Racah's closed form, in exact rational arithmetic
    until the final square root."""
    if m1 + m2 + m3 != 0 or j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    f = math.factorial
    tri = Fraction(f(j1 + j2 - j3) * f(j1 - j2 + j3) * f(-j1 + j2 + j3), f(j1 + j2 + j3 + 1))
    rad = tri * f(j1 + m1) * f(j1 - m1) * f(j2 + m2) * f(j2 - m2) * f(j3 + m3) * f(j3 - m3)
    tmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    tmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = Fraction(0)
    for t in range(tmin, tmax + 1):
        s += Fraction((-1) ** t, f(t) * f(j3 - j2 + t + m1) * f(j3 - j1 + t - m2) * f(j1 + j2 - j3 - t)
                      * f(j1 - t - m1) * f(j2 - t + m2))
    sign = -1 if (j1 - j2 - m3) % 2 else 1
    return sign * float(s) * math.sqrt(float(rad))


def gaunt_yyy(l1, m1, l2, m2, l3, m3):
    """Integral of Y_l1^m1 Y_l2^m2 Y_l3^m3 over the sphere (3j product form)."""
    return (math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4.0 * math.pi))
            * wigner3j(l1, l2, l3, 0, 0, 0) * wigner3j(l1, l2, l3, m1, m2, m3))


def gaunt(n1, m1, l, mu, n, m):
    """Integral of conj(Y_n1^m1) Y_l^mu Y_n^m; conj(Y_a^b) = (-1)^b Y_a^-b."""
    if mu != m1 - m:
        return 0.0
    return (-1) ** (m1 % 2) * gaunt_yyy(n1, -m1, l, mu, n, m)


@lru_cache(maxsize=None)
def _gaunt_table(p_out, p_in):
    """Dense Gaunt(n', m'; l, m' - m; n, m) over (n'm', nm, l)."""
    Lmax = p_out + p_in
    G = np.zeros(((p_out + 1) ** 2, (p_in + 1) ** 2, Lmax + 1))
    for n1 in range(p_out + 1):
        for m1 in range(-n1, n1 + 1):
            for n in range(p_in + 1):
                for m in range(-n, n + 1):
                    mu = m1 - m
                    for l in range(abs(n1 - n), n1 + n + 1):
                        if (n1 + n + l) % 2 or abs(mu) > l:
                            continue
                        G[_cidx(n1, m1), _cidx(n, m), l] = gaunt(n1, m1, l, mu, n, m)
    return G


def translation(t, k, p_out, p_in, kind):
    """Matrix T with coefficients_out = T @ coefficients_in for the shift t:
    kind 'RR' (f_l = j_l: M2M and L2L) or 'SR' (f_l = h_l: M2L)."""
    t = np.asarray(t, dtype=np.float64)
    Lmax = p_out + p_in
    r, th, ph = _sph(t[None, :])
    f = _radial(Lmax, k * r, "j" if kind == "RR" else "h")[0]
    Y = _Y(Lmax, th, ph)[0]
    G = _gaunt_table(p_out, p_in)
    n1 = np.array([n for n in range(p_out + 1) for _ in range(2 * n + 1)])
    m1 = np.array([m for n in range(p_out + 1) for m in range(-n, n + 1)])
    n0 = np.array([n for n in range(p_in + 1) for _ in range(2 * n + 1)])
    m0 = np.array([m for n in range(p_in + 1) for m in range(-n, n + 1)])
    mu = m1[:, None] - m0[None, :]
    T = np.zeros(((p_out + 1) ** 2, (p_in + 1) ** 2), dtype=np.complex128)
    for l in range(Lmax + 1):
        ok = np.abs(mu) <= l
        idx = np.where(ok, l * l + l + mu, 0)
        phase = 1j ** ((n1[:, None] + l - n0[None, :]) % 4)
        T += np.where(ok, phase * f[idx] * np.conj(Y[idx]) * G[:, :, l], 0.0)
    return 4.0 * math.pi * T


# ------------------------------------------------------------------ expansions
def p2m(pts, q, c, k, p):
    """M_nm = i k sum_j q_j conj(R_n^m(y_j - c))."""
    return 1j * k * (np.asarray(q, dtype=np.complex128) @ np.conj(basis_R(p, np.asarray(pts) - c, k)))


def p2l(y, q, c, k, p):
    """Local expansion about c of one source q at y (|x - c| < |y - c|)."""
    d = np.asarray(y, dtype=np.float64) - c
    r, th, ph = _sph(d[None, :])
    return 1j * k * q * _radial(p, k * r, "h")[0] * np.conj(_Y(p, th, ph)[0])


def m2p(M, x, c, k, p):
    """Far field sum M_nm S_n^m(x - c)."""
    return basis_S(p, np.asarray(x) - c, k) @ M


def l2p(L, x, c, k, p):
    """phi(x) = sum L_nm R_n^m(x - c)."""
    return basis_R(p, np.asarray(x) - c, k) @ L


# ------------------------------------------------------------------ the FMM
def fmm3_apply(xyz, q, k, p, leaf, origin=(0.0, 0.0, 0.0), side=1.0, return_parts=False):
    """phi_i = sum_{j != i} G(|x_i - x_j|) q_j by the FMM of Sec. 5.1.2 on the
    uniform oct-tree (readings in the module docstring).  Plain loops over
    boxes and offsets; sizes of a few thousand points."""
    xyz = np.asarray(xyz, dtype=np.float64)
    q = np.asarray(q, dtype=np.complex128)
    o = np.asarray(origin, dtype=np.float64)
    N = len(xyz)
    L = tree_depth3(N, leaf)
    if L == 0:
        near = direct_sum3(xyz, q, k)
        return (near, {"near": near, "far": np.zeros_like(near)}) if return_parts else near
    orders = level_orders3(k, p, L, side)
    nbL = 2 ** L
    s_leaf = side / nbL
    ib = np.clip(np.floor((xyz - o) / s_leaf).astype(np.int64), 0, nbL - 1)

    def lin(i, nb):
        return (i[..., 2] * nb + i[..., 1]) * nb + i[..., 0]

    def centre(i, l):
        return o + (np.asarray(i, dtype=np.float64) + 0.5) * (side / 2 ** l)

    leaf_of = lin(ib, nbL)
    members = [[] for _ in range(nbL ** 3)]
    for j, b in enumerate(leaf_of):
        members[b].append(j)
    members = [np.asarray(mb, dtype=np.int64) for mb in members]

    def unlin(b, nb):
        return np.array([b % nb, (b // nb) % nb, b // (nb * nb)])

    # upward pass
    M = [None] * (L + 1)
    P = [(orders[l] + 1) ** 2 for l in range(L + 1)]
    M[L] = np.zeros((nbL ** 3, P[L]), dtype=np.complex128)
    for b in range(nbL ** 3):
        if len(members[b]):
            M[L][b] = p2m(xyz[members[b]], q[members[b]], centre(unlin(b, nbL), L), k, orders[L])
    for l in range(L - 1, 1, -1):
        nb = 2 ** l
        M[l] = np.zeros((nb ** 3, P[l]), dtype=np.complex128)
        for oc in range(8):
            dc = np.array([oc & 1, (oc >> 1) & 1, (oc >> 2) & 1])
            # child centre minus parent centre = (dc - 1/2) * child side
            t = -(dc - 0.5) * (side / 2 ** (l + 1))
            T = translation(t, k, orders[l], orders[l + 1], "RR")
            for b in range(nb ** 3):
                ch = lin(2 * unlin(b, nb) + dc, 2 * nb)
                M[l][b] += T @ M[l + 1][ch]

    # interaction lists
    Lc = [None] * (L + 1)
    for l in range(2, L + 1):
        nb = 2 ** l
        Lc[l] = np.zeros((nb ** 3, P[l]), dtype=np.complex128)
        cache = {}
        for b in range(nb ** 3):
            it = unlin(b, nb)
            for d in interaction_offsets(tuple(int(v) for v in it % 2)):
                sidx = it - np.asarray(d)
                if np.any(sidx < 0) or np.any(sidx >= nb):
                    continue
                if d not in cache:
                    cache[d] = translation(np.asarray(d, dtype=np.float64) * (side / nb), k, orders[l], orders[l], "SR")
                Lc[l][b] += cache[d] @ M[l][lin(sidx, nb)]

    # downward pass
    for l in range(3, L + 1):
        nb = 2 ** l
        for oc in range(8):
            dc = np.array([oc & 1, (oc >> 1) & 1, (oc >> 2) & 1])
            t = (dc - 0.5) * (side / nb)
            T = translation(t, k, orders[l], orders[l - 1], "RR")
            for b in range(nb ** 3 // 8):
                pi = unlin(b, nb // 2)
                Lc[l][lin(2 * pi + dc, nb)] += T @ Lc[l - 1][b]

    far = np.zeros(N, dtype=np.complex128)
    near = np.zeros(N, dtype=np.complex128)
    for b in range(nbL ** 3):
        tm = members[b]
        if not len(tm):
            continue
        it = unlin(b, nbL)
        far[tm] = l2p(Lc[L][b], xyz[tm], centre(it, L), k, orders[L])
        src = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    jn = it + np.array([dx, dy, dz])
                    if np.all(jn >= 0) and np.all(jn < nbL):
                        src.append(members[lin(jn, nbL)])
        src = np.concatenate(src)
        near[tm] = direct_sum3(xyz[src], q[src], k, targets=xyz[tm])
    phi = near + far
    if return_parts:
        return phi, {"near": near, "far": far, "orders": orders, "L": L}
    return phi
