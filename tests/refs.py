"""Independent numpy references used to pin the oracle.

Nothing here is shared with the oracle or the HIP library: operator tables
come from numpy's Gauss-Legendre rule and numpy polynomial algebra, and each
scheme is written separately from its textbook / paper definition:

* fv_rhs        - first-order finite volumes with an HLL-Einfeldt flux (Sec. 2.1)
* dgsem_rhs     - nodal Gauss DGSEM weak form (Sec. 2.2), mapped to subcell
                  means by the projection (Sec. 2.3), on elements of n subcells
* ml1d_rhs      - the 1-D multi-level blended scheme written in the paper's
                  matrix notation (Sec. 2.6): block-diagonal reconstructions,
                  subcell-interface interpolation, cascade of interface values,
                  common flux and the blended level right-hand sides.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import polynomial as npp

GAMMA = 1.4


def np_tables(n: int, lobatto: bool = False) -> dict:
    if lobatto:
        N = n - 1
        c = np.zeros(N + 1)
        c[-1] = 1.0
        inner = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
        x = np.concatenate([[-1.0], np.sort(inner), [1.0]])
        w = 2.0 / (N * (N + 1) * np.polynomial.legendre.legval(x, c) ** 2)
    else:
        x, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * x, 0.5 * w
    basis = []
    for j in range(n):
        cj = npp.polyfromroots(np.delete(x, j))
        basis.append(cj / npp.polyval(x[j], cj))
    Dcal = np.array([[npp.polyval(x[i], npp.polyder(basis[j])) for j in range(n)] for i in range(n)])
    P = np.zeros((n, n))
    for j in range(n):
        F = npp.polyint(basis[j])
        for i in range(n):
            a, b = -0.5 + i / n, -0.5 + (i + 1) / n
            P[i, j] = n * (npp.polyval(b, F) - npp.polyval(a, F))
    R = np.linalg.inv(P)
    bm = np.array([npp.polyval(-0.5, basis[j]) for j in range(n)])
    bp = np.array([npp.polyval(0.5, basis[j]) for j in range(n)])
    D = np.diag(1.0 / w) @ Dcal.T @ np.diag(w)
    Ip = np.array([[npp.polyval(-0.5 + (i + 1) / n, basis[j]) for j in range(n)] for i in range(n)])
    Im = np.array([[npp.polyval(-0.5 + i / n, basis[j]) for j in range(n)] for i in range(n)])
    return dict(x=x, w=w, Dcal=Dcal, D=D, P=P, R=R, bm=bm, bp=bp, Ip=Ip, Im=Im, basis=basis)


# ---------------------------------------------------------------------------
# Euler physics, vectorised over trailing axes; state axis 0 = variables
# ---------------------------------------------------------------------------

def pressure(u, dim, g=GAMMA):
    m2 = sum(u[1 + a] ** 2 for a in range(dim))
    return (g - 1.0) * (u[dim + 1] - 0.5 * m2 / u[0])


def flux(u, dim, a, g=GAMMA):
    p = pressure(u, dim, g)
    va = u[1 + a] / u[0]
    f = np.empty_like(u)
    f[0] = u[1 + a]
    for b in range(dim):
        f[1 + b] = u[1 + b] * va + (p if a == b else 0.0)
    f[dim + 1] = va * (u[dim + 1] + p)
    return f


def hlle(uL, uR, dim, a, g=GAMMA):
    """HLL flux with Einfeldt wave speeds (Roe averages)."""
    fL, fR = flux(uL, dim, a, g), flux(uR, dim, a, g)
    pL, pR = pressure(uL, dim, g), pressure(uR, dim, g)
    cL, cR = np.sqrt(g * pL / uL[0]), np.sqrt(g * pR / uR[0])
    sL, sR = np.sqrt(uL[0]), np.sqrt(uR[0])
    vel = [(sL * uL[1 + b] / uL[0] + sR * uR[1 + b] / uR[0]) / (sL + sR) for b in range(dim)]
    H = (sL * (uL[dim + 1] + pL) / uL[0] + sR * (uR[dim + 1] + pR) / uR[0]) / (sL + sR)
    c = np.sqrt((g - 1.0) * (H - 0.5 * sum(v * v for v in vel)))
    SL = np.minimum(uL[1 + a] / uL[0] - cL, vel[a] - c)
    SR = np.maximum(uR[1 + a] / uR[0] + cR, vel[a] + c)
    SLm, SRp = np.minimum(SL, 0.0), np.maximum(SR, 0.0)
    return (SRp * fL - SLm * fR + SLm * SRp * (uR - uL)) / (SRp - SLm)


# ---------------------------------------------------------------------------
# helpers on the global grid u[v, z, y, x] (dim-generic with numpy axes)
# ---------------------------------------------------------------------------

def _axis(dim, a):
    """numpy axis of spatial axis a in an array shaped (nv, Gz, Gy, Gx)."""
    return 3 - a


def _neighbours(u, a, bc):
    """Left and right neighbour copies along spatial axis a (periodic or outflow)."""
    ax = 3 - a
    if bc == 0:
        return np.roll(u, 1, axis=ax), np.roll(u, -1, axis=ax)
    n = u.shape[ax]
    idxl = np.concatenate([[0], np.arange(n - 1)])
    idxr = np.concatenate([np.arange(1, n), [n - 1]])
    return np.take(u, idxl, axis=ax), np.take(u, idxr, axis=ax)


def fv_rhs(mesh, u):
    """First-order subcell finite volumes: -(1/h_a) (f*_{i+1/2} - f*_{i-1/2})."""
    dim = mesh.dim
    ne, lo, hi, bc = mesh.full()
    out = np.zeros_like(u)
    for a in range(dim):
        h = (hi[a] - lo[a]) / (ne[a] * mesh.K)
        ul, ur = _neighbours(u, a, bc[a])
        fright = hlle(u, ur, dim, a)
        fleft = hlle(ul, u, dim, a)
        out -= (fright - fleft) / h
    return out


def _to_blocks(u, dim, n):
    """(nv, Gz, Gy, Gx) -> (nv, Ez, n, Ey, n, Ex, n) with unit extents for unused axes."""
    nv, gz, gy, gx = u.shape
    nz = n if dim > 2 else 1
    ny = n if dim > 1 else 1
    return u.reshape(nv, gz // nz, nz, gy // ny, ny, gx // n, n)


def _from_blocks(b):
    nv, ez, nz, ey, ny, ex, nx = b.shape
    return b.reshape(nv, ez * nz, ey * ny, ex * nx)


def _apply(b, M, a, dim):
    """Apply matrix M along local node axis of spatial axis a in block layout."""
    ax = {0: 6, 1: 4, 2: 2}[a]
    return np.moveaxis(np.tensordot(M, b, axes=([1], [ax])), 0, ax)


def dgsem_rhs(mesh, ubar, n, tabs=None):
    """Nodal Gauss DGSEM on elements of n^dim subcells (element width n/K of a
    mesh element), HLLE surface flux, then mapped to subcell means: returns
    d(ubar)/dt = P^{(x)dim} applied to the nodal right-hand side."""
    dim = mesh.dim
    T = tabs or np_tables(n)
    ne, lo, hi, bc = mesh.full()
    b = _to_blocks(ubar, dim, n)
    ut = b
    for a in range(dim):
        ut = _apply(ut, T["R"], a, dim)
    out = np.zeros_like(ut)
    Bl = -T["bm"] / T["w"]
    Br = T["bp"] / T["w"]
    for a in range(dim):
        h = (hi[a] - lo[a]) / (ne[a] * mesh.K) * n
        f = flux(ut, dim, a)
        vol = _apply(f, T["D"], a, dim)
        ax = {0: 6, 1: 4, 2: 2}[a]
        eax = ax - 1
        tr_m = np.tensordot(ut, T["bm"], axes=([ax], [0]))  # element left-face trace
        tr_p = np.tensordot(ut, T["bp"], axes=([ax], [0]))  # element right-face trace
        eax_t = eax  # element axis index unchanged (contracted axis was after it)
        nE = tr_m.shape[eax_t]
        if bc[a] == 0:
            left_nb = np.roll(tr_p, 1, axis=eax_t)
            right_nb = np.roll(tr_m, -1, axis=eax_t)
        else:
            il = np.concatenate([[0], np.arange(nE - 1)])
            ir = np.concatenate([np.arange(1, nE), [nE - 1]])
            left_nb = np.take(tr_p, il, axis=eax_t)
            right_nb = np.take(tr_m, ir, axis=eax_t)
            # outflow: the exterior state is the boundary subcell's mean (zero gradient of the
            # subcell means), nodal along the face
            bt = b
            for c2 in range(dim):
                if c2 != a:
                    bt = _apply(bt, T["R"], c2, dim)
            g_lo = np.take(bt, 0, axis=ax)
            g_hi = np.take(bt, bt.shape[ax] - 1, axis=ax)
            sl = [slice(None)] * tr_m.ndim
            sl[eax_t] = 0
            left_nb[tuple(sl)] = g_lo[tuple(sl)]
            sl[eax_t] = nE - 1
            right_nb[tuple(sl)] = g_hi[tuple(sl)]
        fl = hlle(left_nb, tr_m, dim, a)
        fr = hlle(tr_p, right_nb, dim, a)
        surf = np.expand_dims(fl, ax) * Bl.reshape([-1 if i == ax else 1 for i in range(ut.ndim)]) + \
            np.expand_dims(fr, ax) * Br.reshape([-1 if i == ax else 1 for i in range(ut.ndim)])
        out += (vol - surf) / h
    for a in range(dim):
        out = _apply(out, T["P"], a, dim)
    return _from_blocks(out)


# ---------------------------------------------------------------------------
# 1-D multi-level blended scheme in the paper's matrix notation (Sec. 2.6)
# ---------------------------------------------------------------------------

def _blockdiag(M, reps):
    return np.kron(np.eye(reps), M)


def ml1d_rhs(K, nelem, dx, ubar, alphas, levels, periodic=True, g=GAMMA):
    """ubar: (3, nelem*K).  alphas: dict level n -> array (nelem, K//n).
    Squeezing is not modelled: every reconstruction must be permissible at its
    nodes and sub-element boundaries (the caller checks that beta = 1)."""
    dim = 1
    nv = 3
    U = ubar.reshape(nv, nelem, K)
    tabs = {n: np_tables(n) for n in levels}
    # interface values per element: u^{+-}(n) (length K each), cascade in alpha (Sec. 2.6)
    up = U.copy()   # level O(1): u^{+-O(1)} = means
    um = U.copy()
    levels_lo = sorted(levels)  # 2, 4, ..., K: cascade from lowest to highest order
    recon = {}
    for n in levels_lo:
        T = tabs[n]
        Rb = _blockdiag(T["R"], K // n)
        ut = np.einsum("ij,vej->vei", Rb, U)
        recon[n] = ut
        Ipb = _blockdiag(T["Ip"], K // n)
        Imb = _blockdiag(T["Im"], K // n)
        upn = np.einsum("ij,vej->vei", Ipb, ut)
        umn = np.einsum("ij,vej->vei", Imb, ut)
        al = np.repeat(alphas[n], n, axis=1)[None]
        up = (1.0 - al) * up + al * upn
        um = (1.0 - al) * um + al * umn
    # append neighbours: u+ = ((u+_K)_{q-1}, u+_1..u+_K); u- = (u-_1..u-_K, (u-_1)_{q+1})
    if periodic:
        left = np.roll(up[:, :, K - 1], 1, axis=1)
        right = np.roll(um[:, :, 0], -1, axis=1)
    else:
        # outflow: the exterior state is the boundary subcell's mean
        left = up[:, :, K - 1].copy()
        left[:, 1:] = up[:, :-1, K - 1]
        left[:, 0] = U[:, 0, 0]
        right = um[:, :, 0].copy()
        right[:, :-1] = um[:, 1:, 0]
        right[:, -1] = U[:, -1, K - 1]
    Up = np.concatenate([left[:, :, None], up], axis=2)       # (nv, nelem, K+1)
    Um = np.concatenate([um, right[:, :, None]], axis=2)
    fstar = hlle(Up, Um, dim, 0, g)                           # (nv, nelem, K+1)
    # level right-hand sides
    Delta = np.zeros((K, K + 1))
    for i in range(K):
        Delta[i, i], Delta[i, i + 1] = -1.0, 1.0
    rhs = {1: -(K / dx) * np.einsum("ij,vej->vei", Delta, fstar)}
    for n in levels_lo:
        T = tabs[n]
        Dhat = T["P"] @ T["D"]
        B0 = np.zeros((n, n + 1))
        B0[:, 0] = -T["bm"] / T["w"]
        B0[:, n] = T["bp"] / T["w"]
        Bhat = T["P"] @ B0
        # [I_{K/n} (x) Bhat]^(0): K x (K+1), sub-element s uses columns s*n and (s+1)*n
        Bbig = np.zeros((K, K + 1))
        for s in range(K // n):
            Bbig[s * n:(s + 1) * n, s * n] = Bhat[:, 0]
            Bbig[s * n:(s + 1) * n, (s + 1) * n] = Bhat[:, n]
        ft = flux(recon[n], dim, 0, g)
        vol = np.einsum("ij,vej->vei", _blockdiag(Dhat, K // n), ft)
        rhs[n] = (K / (n * dx)) * (vol - np.einsum("ij,vej->vei", Bbig, fstar))
    # blend from the lowest to the highest order (eq. multilevel-blending-discretizations)
    acc = rhs[1]
    for n in levels_lo:
        al = np.repeat(alphas[n], n, axis=1)[None]
        acc = (1.0 - al) * acc + al * rhs[n]
    return acc.reshape(nv, nelem * K)


def ml2d_rhs(K, ne, dx, ubar, alpha, levels, g=GAMMA):
    """Dense brute force of the 2-D multi-level blended scheme on a periodic mesh of
    ne x ne square elements of width dx (Sec. 2.6 in two dimensions; App. eqs.
    3D-interface-fluxes and 3D-blend-interface-fluxes reduced to d = 2).

    ubar: (4, G, G) subcell means indexed [v, y, x], G = ne*K.  alpha: (ne*ne, A)
    per element (x fastest), levels listed from the top (K, K/2, ..., 2), level n's
    sub-elements at offsets sum_{m > n} (K/m)^2, x fastest inside the element.
    Every operator is a dense G x G matrix on one global axis, block-diagonal over
    the level-n sub-elements (Kronecker product with the identity).  Squeezing and the
    interface safety rule are not modelled: the caller checks that neither acts."""
    dim, nv, G = 2, 4, ne * K
    U = ubar
    tabs = {n: np_tables(n) for n in levels}

    def blk(M, n):
        return np.kron(np.eye(G // n), M)

    def along(X, M, a):          # contract M with spatial axis a (0 = x, 1 = y)
        return np.einsum("ij,vyj->vyi", M, X) if a == 0 else np.einsum("ij,vjx->vix", M, X)

    # per-cell blending weights (eq. blending-weights)
    iy, ix = np.meshgrid(np.arange(G), np.arange(G), indexing="ij")
    elem = (ix // K) + ne * (iy // K)
    th, prod, off = {}, np.ones((G, G)), 0
    for n in levels:
        ns = K // n
        a_n = alpha[elem, off + (ix % K) // n + ns * ((iy % K) // n)]
        th[n] = a_n * prod
        prod = prod * (1.0 - a_n)
        off += ns * ns
    th1 = prod

    rhs = {1: np.zeros_like(U)}
    rhs.update({n: np.zeros_like(U) for n in levels})
    nodal = {n: along(along(U, blk(tabs[n]["R"], n), 0), blk(tabs[n]["R"], n), 1) for n in levels}
    for a in range(dim):
        b = 1 - a
        # interface states of every cell at its high (+) and low (-) face along a: cascade
        up, um = th1[None] * U, th1[None] * U
        for n in levels:
            T = tabs[n]
            up = up + th[n][None] * along(U, blk(T["Ip"] @ T["R"], n), a)
            um = um + th[n][None] * along(U, blk(T["Im"] @ T["R"], n), a)
        # face f along a lies between cell f-1 (left) and cell f (right), periodic
        ax = 2 - a
        uL = np.roll(up, 1, axis=ax)
        uR = um
        F = hlle(uL, uR, dim, a, g)
        wsum = np.zeros((G, G))
        acc = np.zeros_like(U)
        fidx = np.arange(G)
        for n in levels:
            T = tabs[n]
            cand = along(hlle(along(uL, blk(T["R"], n), b), along(uR, blk(T["R"], n), b), dim, a, g),
                         blk(T["P"], n), b)
            tbar = 0.5 * (np.roll(th[n], 1, axis=ax - 1) + th[n])
            on = (fidx % n == 0)
            mask = on[None, :] if a == 0 else on[:, None]
            wn = np.where(mask, tbar, 0.0)
            acc = acc + wn[None] * cand
            wsum = wsum + wn
        F = acc + (1.0 - wsum)[None] * F
        # first-order finite volumes
        rhs[1] = rhs[1] - (K / dx) * (np.roll(F, -1, axis=ax) - F)
        # DG levels: (K / (n dx)) (f(nodal) x_a Dhat x_b P - F* x_a Bhat)
        for n in levels:
            T = tabs[n]
            Dhat = T["P"] @ T["D"]
            B0 = np.zeros((n, n + 1))
            B0[:, 0] = -T["bm"] / T["w"]
            B0[:, n] = T["bp"] / T["w"]
            Bhat = T["P"] @ B0
            Bbig = np.zeros((G, G))
            for s in range(G // n):
                Bbig[s * n:(s + 1) * n, s * n] += Bhat[:, 0]
                Bbig[s * n:(s + 1) * n, ((s + 1) * n) % G] += Bhat[:, n]
            vol = along(along(flux(nodal[n], dim, a, g), blk(Dhat, n), a), blk(T["P"], n), b)
            rhs[n] = rhs[n] + (K / (n * dx)) * (vol - along(F, Bbig, a))
    out = th1[None] * rhs[1]
    for n in levels:
        out = out + th[n][None] * rhs[n]
    return out
