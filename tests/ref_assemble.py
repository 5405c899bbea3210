"""Brute-force dense assembly of the weighted SIPG operator, for tiny meshes.

An independent second route to the matrix of eq. (blf) (Sec. 2.2): numpy only,
basis values from ``numpy.polynomial.legendre`` (not from the oracle), Gauss
nodes from ``numpy.polynomial.legendre.leggauss``, and the face terms written
generically in jump/average form for every (trial side, test side) pair instead
of the per-side expansions the oracle uses.  Dense matrices: a few hundred DOF
at most.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


def _basis_1d(k: int, t: np.ndarray):
    """theta_j(t) = sqrt(2j+1) P_j(2t-1) and its t-derivative, shape (len(t), k+1)."""
    s = 2.0 * np.asarray(t, dtype=np.float64) - 1.0
    V = np.empty((s.size, k + 1))
    D = np.empty((s.size, k + 1))
    for j in range(k + 1):
        c = np.zeros(j + 1)
        c[j] = np.sqrt(2 * j + 1)
        V[:, j] = L.legval(s, c)
        D[:, j] = 2.0 * L.legval(s, L.legder(c))
    return V, D


def _gauss01(m: int):
    x, w = L.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def _tensor_shape(vals, ders, h):
    """Given per-axis (npts_a, n) value/derivative tables on a tensor grid of
    points, return phi (P, n^3) and grad (P, n^3, 3) with axis 1 fastest in both
    the point and the shape-function numbering."""
    n = vals[0].shape[1]
    P = [v.shape[0] for v in vals]
    phi = np.einsum("ai,bj,ck->cbakji", vals[0], vals[1], vals[2]).reshape(P[0] * P[1] * P[2], n ** 3)
    g1 = np.einsum("ai,bj,ck->cbakji", ders[0], vals[1], vals[2]).reshape(-1, n ** 3) / h[0]
    g2 = np.einsum("ai,bj,ck->cbakji", vals[0], ders[1], vals[2]).reshape(-1, n ** 3) / h[1]
    g3 = np.einsum("ai,bj,ck->cbakji", vals[0], vals[1], ders[2]).reshape(-1, n ** 3) / h[2]
    return phi, np.stack([g1, g2, g3], axis=-1)


def _b(prob, X):
    b = np.empty_like(X)
    amp = getattr(prob, "b_amp", None)
    for r in range(3):
        if amp is None:
            b[:, r] = prob.b_const[r] + prob.b_sin[r] * np.sin(np.pi * X[:, prob.b_axis[r]])
        else:
            b[:, r] = amp[r]
            for j in range(3):
                w = prob.b_freq[3 * r + j]
                if w != 0.0:
                    b[:, r] *= np.sin(w * X[:, j] + prob.b_phase[3 * r + j])
    return b


def _kp(prob, X):
    """Polynomial diffusion factor prod_j (c0 + c1 x_j + c2 x_j^2) at points X (1 if unset)."""
    c = getattr(prob, "kappa_poly", None)
    if c is None:
        return np.ones(X.shape[0])
    v = np.ones(X.shape[0])
    for j in range(3):
        v *= c[3 * j] + c[3 * j + 1] * X[:, j] + c[3 * j + 2] * X[:, j] ** 2
    return v


def assemble_dense(prob) -> np.ndarray:
    k = prob.k
    n = k + 1
    nb = n ** 3
    N = prob.ncell
    nc = N[0] * N[1] * N[2]
    A = np.zeros((nc * nb, nc * nb))
    xi, w = _gauss01(k + 1 + int(getattr(prob, "quad_extra", 0)))
    Vq, Dq = _basis_1d(k, xi)
    V0, D0 = _basis_1d(k, np.array([0.0]))
    V1, D1 = _basis_1d(k, np.array([1.0]))
    K = np.asarray(prob.K, dtype=np.float64)
    kap = np.ones(nc) if prob.kappa is None else np.asarray(prob.kappa).ravel()
    # affine map x = A xi of the tensor grid: gradients A^{-T} grad_xi, measures |det A|
    Aff = getattr(prob, "affine", None)
    Aff = np.eye(3) if Aff is None else np.asarray(Aff, dtype=np.float64).reshape(3, 3)
    AiT = np.linalg.inv(Aff).T
    detA = abs(np.linalg.det(Aff))

    def phys(g):
        return np.einsum("rs,pjs->pjr", AiT, g)

    def cid(i):
        return i[0] + N[0] * (i[1] + N[1] * i[2])

    def geom(i):
        o = np.array([prob.nodes[a][i[a]] for a in range(3)])
        h = np.array([prob.nodes[a][i[a] + 1] - prob.nodes[a][i[a]] for a in range(3)])
        return o, h

    def blk(c):
        return slice(c * nb, (c + 1) * nb)

    cells = [(i1, i2, i3) for i3 in range(N[2]) for i2 in range(N[1]) for i1 in range(N[0])]
    # ---- volume: (D grad u - b u, grad v)_T + (c u, v)_T ----
    for i in cells:
        o, h = geom(i)
        c = cid(i)
        phi, g = _tensor_shape([Vq] * 3, [Dq] * 3, h)
        g = phys(g)
        Wq = np.einsum("a,b,c->cba", w, w, w).ravel() * np.prod(h) * detA
        Xi = np.stack(np.meshgrid(o[0] + h[0] * xi, o[1] + h[1] * xi, o[2] + h[2] * xi,
                                  indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
        Xq = Xi @ Aff.T                     # physical points (b); kp at the grid points Xi
        bq = _b(prob, Xq)
        Dg = kap[c] * _kp(prob, Xi)[:, None, None] * np.einsum("rs,pjs->pjr", K, g)  # D grad phi_j
        flux = Dg - bq[:, None, :] * phi[:, :, None]              # (P, j, 3)
        A[blk(c), blk(c)] += np.einsum("p,pjr,pir->ij", Wq, flux, g)
        A[blk(c), blk(c)] += prob.c * np.einsum("p,pj,pi->ij", Wq, phi, phi)

    # ---- faces ----
    def face_tables(a, e, h):
        """phi, grad on the face x_a = e (reference) at tangential Gauss nodes."""
        vals, ders = [Vq, Vq, Vq], [Dq, Dq, Dq]
        vals = list(vals)
        ders = list(ders)
        vals[a] = V1 if e == 1 else V0
        ders[a] = D1 if e == 1 else D0
        ph, gr = _tensor_shape(vals, ders, h)
        return ph, phys(gr)

    def face_weights(a, h):
        ws = [w, w, w]
        ws[a] = np.array([1.0])
        W = np.einsum("a,b,c->cba", ws[0], ws[1], ws[2]).ravel()
        t = [b for b in range(3) if b != a]
        return W * h[t[0]] * h[t[1]]

    def face_points(a, o, h, xa):
        """grid points of the face and their physical images"""
        pts = [o[b] + h[b] * xi for b in range(3)]
        pts[a] = np.array([xa])
        G = np.stack(np.meshgrid(*pts, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
        return G, G @ Aff.T

    def normal(a):
        """unit normal A^{-T} e_a / |A^{-T} e_a| and |A^{-T} e_a|"""
        v = AiT[:, a]
        return v / np.linalg.norm(v), np.linalg.norm(v)

    per = getattr(prob, "periodic", (False, False, False))
    for i in cells:
        for a in range(3):
            o, h = geom(i)
            c = cid(i)
            if i[a] + 1 < N[a] or per[a]:
                # on a periodic axis the last cell's upper face meets the first
                # cell, whose lower node carries the face's velocity
                ip = list(i)
                ip[a] = (i[a] + 1) % N[a]
                op, hp = geom(ip)
                cp = cid(ip)
                nu, nrm = normal(a)
                W = face_weights(a, h) * detA * nrm
                Xg, X = face_points(a, o, h, op[a])
                bnu = _b(prob, X) @ nu
                kpf = _kp(prob, Xg)                     # pointwise diffusion factor (grid coordinates)
                Knn = nu @ K @ nu
                dm, dp = kap[c] * kpf * Knn, kap[cp] * kpf * Knn
                wm, wp = dp / (dm + dp), dm / (dm + dp)
                gam = prob.sigma * (2 * dm * dp / (dm + dp)) * nrm / min(h[a], hp[a])
                side = {0: (c, *face_tables(a, 1, h), kap[c] * kpf), 1: (cp, *face_tables(a, 0, hp), kap[cp] * kpf)}
                for su in (0, 1):        # trial function side (0: minus, 1: plus)
                    for sv in (0, 1):    # test function side
                        cu, phu, gu, ku = side[su]
                        cv, phv, gv, kv = side[sv]
                        um = phu if su == 0 else 0 * phu
                        up = phu if su == 1 else 0 * phu
                        jump_u = um - up
                        avg_u = ((wm if su == 0 else wp) * ku)[:, None] * np.einsum("s,pjs->pj", nu @ K, gu)
                        Phi = np.where(bnu[:, None] >= 0, bnu[:, None] * um, bnu[:, None] * up)
                        jump_v = phv if sv == 0 else -phv
                        avg_v = ((wm if sv == 0 else wp) * kv)[:, None] * np.einsum("s,pis->pi", nu @ K, gv)
                        M = (np.einsum("p,pj,pi->ij", W, Phi, jump_v)
                             - np.einsum("p,pj,pi->ij", W, avg_u, jump_v)
                             - np.einsum("p,pi,pj->ij", W, avg_v, jump_u)
                             + np.einsum("p,pj,pi->ij", W * gam, jump_u, jump_v))
                        A[blk(cv), blk(cu)] += M
            for e in (0, 1):
                at_bnd = (i[a] == 0) if e == 0 else (i[a] == N[a] - 1)
                if not at_bnd or per[a]:
                    continue
                nu, nrm = normal(a)
                W = face_weights(a, h) * detA * nrm
                Xg, X = face_points(a, o, h, o[a] + (h[a] if e == 1 else 0.0))
                nsg = 1.0 if e == 1 else -1.0
                bnu = nsg * (_b(prob, X) @ nu)
                kpf = _kp(prob, Xg)
                delta = kap[c] * kpf * (nu @ K @ nu)
                gam = prob.sigma * delta * nrm / h[a]
                ph, g = face_tables(a, e, h)
                Dn = nsg * (kap[c] * kpf)[:, None] * np.einsum("s,pjs->pj", nu @ K, g)
                Phi = np.where(bnu[:, None] >= 0, bnu[:, None] * ph, 0.0)
                M = (np.einsum("p,pj,pi->ij", W, Phi, ph)
                     - np.einsum("p,pj,pi->ij", W, Dn, ph)
                     - np.einsum("p,pi,pj->ij", W, Dn, ph)
                     + np.einsum("p,pj,pi->ij", W * gam, ph, ph))
                A[blk(c), blk(c)] += M
    return A


# ---------------------------------------------------------------------------
# Multilinear geometry: every cell the trilinear image of [0,1]^3 through its
# eight vertices, the geometry evaluated point by point.  Written separately
# from the tensor-grid assembly above and from the oracle's route: Jacobians
# from numpy differences of the corner weights, gradients through
# numpy.linalg.inv, face normals as cross products of the tangential Jacobian
# columns.
# ---------------------------------------------------------------------------
def _corners(prob, i):
    """The eight vertices of cell i, shape (2, 2, 2, 3) indexed [c0, c1, c2]."""
    V = np.asarray(prob.vertices, dtype=np.float64)  # (N3+1, N2+1, N1+1, 3)
    return V[i[2]:i[2] + 2, i[1]:i[1] + 2, i[0]:i[0] + 2].transpose(2, 1, 0, 3)


def _trilinear(Xc, pts):
    """Points and Jacobians of the trilinear map at reference points pts (P, 3):
    x(xi) = sum_c Xc[c] prod_a l_{c_a}(xi_a); J[p, r, s] = d x_r / d xi_s."""
    l = np.stack([1.0 - pts, pts], axis=1)          # (P, 2, 3): l_c(xi_a)
    dl = np.array([-1.0, 1.0])
    X = np.einsum("pa,pb,pc,abcr->pr", l[:, :, 0], l[:, :, 1], l[:, :, 2], Xc)
    J0 = np.einsum("a,pb,pc,abcr->pr", dl, l[:, :, 1], l[:, :, 2], Xc)
    J1 = np.einsum("pa,b,pc,abcr->pr", l[:, :, 0], dl, l[:, :, 2], Xc)
    J2 = np.einsum("pa,pb,c,abcr->pr", l[:, :, 0], l[:, :, 1], dl, Xc)
    return X, np.stack([J0, J1, J2], axis=-1)


def _ref_points(vals_pts):
    """Tensor points (axis 1 fastest) from per-axis coordinate arrays."""
    G = np.stack(np.meshgrid(*vals_pts, indexing="ij"), axis=-1)
    return G.transpose(2, 1, 0, 3).reshape(-1, 3)


def assemble_dense_multilinear(prob) -> np.ndarray:
    k = prob.k
    n = k + 1
    nb = n ** 3
    N = prob.ncell
    nc = N[0] * N[1] * N[2]
    A = np.zeros((nc * nb, nc * nb))
    xi, w = _gauss01(k + 1 + int(getattr(prob, "quad_extra", 0)))
    Vq, Dq = _basis_1d(k, xi)
    V0, D0 = _basis_1d(k, np.array([0.0]))
    V1, D1 = _basis_1d(k, np.array([1.0]))
    K = np.asarray(prob.K, dtype=np.float64)
    kap = np.ones(nc) if prob.kappa is None else np.asarray(prob.kappa).ravel()

    def cid(i):
        return i[0] + N[0] * (i[1] + N[1] * i[2])

    def blk(c):
        return slice(c * nb, (c + 1) * nb)

    def phys(gref, J):
        Jinv = np.linalg.inv(J)                      # (P, 3, 3)
        return np.einsum("psr,pjs->pjr", Jinv, gref)  # J^{-T} grad_ref

    def volume(i):
        _, J = _trilinear(_corners(prob, i), _ref_points([xi, xi, xi]))
        return float(np.einsum("a,b,c->cba", w, w, w).ravel() @ np.linalg.det(J))

    def face(i, a, e):
        """reference points, physical points, Jacobians, area-weighted normal
        (towards increasing xi_a), weights and shape tables of face xi_a = e."""
        t = [b for b in range(3) if b != a]
        pts = [xi, xi, xi]
        pts[a] = np.array([float(e)])
        R = _ref_points(pts)
        X, J = _trilinear(_corners(prob, i), R)
        b_, c_ = (a + 1) % 3, (a + 2) % 3
        nv = np.cross(J[:, :, b_], J[:, :, c_])
        ws = [w, w, w]
        ws[a] = np.array([1.0])
        W = np.einsum("a,b,c->cba", ws[0], ws[1], ws[2]).ravel()
        vals, ders = [Vq, Vq, Vq], [Dq, Dq, Dq]
        vals[a] = V1 if e == 1 else V0
        ders[a] = D1 if e == 1 else D0
        ph, gr = _tensor_shape(vals, ders, np.ones(3))
        return X, J, nv, W, ph, phys(gr, J), t

    cells = [(i1, i2, i3) for i3 in range(N[2]) for i2 in range(N[1]) for i1 in range(N[0])]
    for i in cells:
        c = cid(i)
        X, J = _trilinear(_corners(prob, i), _ref_points([xi, xi, xi]))
        phi, gref = _tensor_shape([Vq] * 3, [Dq] * 3, np.ones(3))
        g = phys(gref, J)
        Wq = np.einsum("a,b,c->cba", w, w, w).ravel() * np.linalg.det(J)
        Dg = kap[c] * _kp(prob, X)[:, None, None] * np.einsum("rs,pjs->pjr", K, g)
        flux = Dg - _b(prob, X)[:, None, :] * phi[:, :, None]
        A[blk(c), blk(c)] += np.einsum("p,pjr,pir->ij", Wq, flux, g)
        A[blk(c), blk(c)] += prob.c * np.einsum("p,pj,pi->ij", Wq, phi, phi)

    for i in cells:
        c = cid(i)
        for a in range(3):
            if i[a] + 1 < N[a]:
                ip = list(i)
                ip[a] += 1
                cp = cid(ip)
                X, Jm, nv, W0, phm, gm, _ = face(i, a, 1)
                _, Jp, _, _, php, gp, _ = face(ip, a, 0)
                nrm = np.linalg.norm(nv, axis=1)
                nu = nv / nrm[:, None]
                W = W0 * nrm
                FoT = float(W0 @ nrm) / min(volume(i), volume(ip))
                bnu = np.einsum("pr,pr->p", _b(prob, X), nu)
                kpf = _kp(prob, X)
                Knn = np.einsum("pr,rs,ps->p", nu, K, nu)
                dm, dp = kap[c] * kpf * Knn, kap[cp] * kpf * Knn
                wm, wp = dp / (dm + dp), dm / (dm + dp)
                gam = prob.sigma * (2 * dm * dp / (dm + dp)) * FoT
                nK = nu @ K
                side = {0: (c, phm, gm, kap[c] * kpf), 1: (cp, php, gp, kap[cp] * kpf)}
                for su in (0, 1):
                    for sv in (0, 1):
                        cu, phu, gu, ku = side[su]
                        cv, phv, gv, kv = side[sv]
                        um = phu if su == 0 else 0 * phu
                        up = phu if su == 1 else 0 * phu
                        jump_u = um - up
                        avg_u = ((wm if su == 0 else wp) * ku)[:, None] * np.einsum("ps,pjs->pj", nK, gu)
                        Phi = np.where(bnu[:, None] >= 0, bnu[:, None] * um, bnu[:, None] * up)
                        jump_v = phv if sv == 0 else -phv
                        avg_v = ((wm if sv == 0 else wp) * kv)[:, None] * np.einsum("ps,pis->pi", nK, gv)
                        M = (np.einsum("p,pj,pi->ij", W, Phi, jump_v)
                             - np.einsum("p,pj,pi->ij", W, avg_u, jump_v)
                             - np.einsum("p,pi,pj->ij", W, avg_v, jump_u)
                             + np.einsum("p,pj,pi->ij", W * gam, jump_u, jump_v))
                        A[blk(cv), blk(cu)] += M
            for e in (0, 1):
                if (i[a] == 0) if e == 0 else (i[a] == N[a] - 1):
                    X, J, nv, W0, ph, g, _ = face(i, a, e)
                    nv = nv if e == 1 else -nv
                    nrm = np.linalg.norm(nv, axis=1)
                    nu = nv / nrm[:, None]
                    W = W0 * nrm
                    FoT = float(W0 @ nrm) / volume(i)
                    bnu = np.einsum("pr,pr->p", _b(prob, X), nu)
                    kx = kap[c] * _kp(prob, X)
                    gam = prob.sigma * kx * np.einsum("pr,rs,ps->p", nu, K, nu) * FoT
                    Dn = kx[:, None] * np.einsum("ps,pjs->pj", nu @ K, g)
                    Phi = np.where(bnu[:, None] >= 0, bnu[:, None] * ph, 0.0)
                    M = (np.einsum("p,pj,pi->ij", W, Phi, ph)
                         - np.einsum("p,pj,pi->ij", W, Dn, ph)
                         - np.einsum("p,pi,pj->ij", W, Dn, ph)
                         + np.einsum("p,pj,pi->ij", W * gam, ph, ph))
                    A[blk(c), blk(c)] += M
    return A
