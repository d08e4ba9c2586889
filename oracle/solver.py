"""DBFFT linear systems, preconditioned CG and Newton (oracle; test
infrastructure only).

Unknown: {a | e}, a the normalized Fourier coefficients of the displacement
fluctuation on the half spectrum (3 components), e the macroscopic strain
(small strains) or displacement-gradient (finite strains) components on the
stress-controlled set S, in an orthonormal basis.

Operator (sign-flipped so that it is positive semi-definite; the printed
operator d:F(C:F^-1(s.u)) is its negative, Sec. 2.2 eq. lineqf):
    eps(x)   = E + sum_a e_a B_a + sum_k (s(k).a(k)) exp(i xi.x)
    sigma(x) = C(x) : eps(x)
    s(k)     = F[sigma](k) / N
    (K{a|e})_a(k) = -i xi_j s_ij(k)  (k outside the null set, else 0)
    (K{a|e})_e    = B_a : s(0) = B_a : <sigma>,   a in S
This is the Hessian of the average energy 1/2 <eps:C:eps> - sbar_S . e, so it
is symmetric for the real inner product on the half spectrum plus the
Euclidean product on e (Sec. 2.2 and Sec. 2.3: full rank and Hermitian once
the zero frequency and the duplicated real-transform terms are removed).

Right-hand side (Sec. 2.2 eq. lineqf, Sec. 2.3 final system):
    b_a = i xi_j F[C:E_U]_ij / N,   b_e = sbar_S - B_a : <C:E_U>.

Preconditioner (Sec. 2.5 eqs. pred2/pred3): M(xi) = [xi.Cbar.xi]^-1 with
(xi.Cbar.xi)_ik = xi_j Cbar_ijkl xi_l, Cbar the voxel average of the
stiffness (or tangent); at xi = 0 the macro block uses [B_a:Cbar:B_b]^-1.

Residuals (Sec. 3, eqs. chedckeq and chedckimp): the equilibrium residual
||div sigma||_L2 / ||<sigma>|| with the L2 norm taken as the RMS over the
unit cell equals the full-spectrum norm of the a-part of the CG residual
divided by ||<sigma>||_F; the loading residual is ||r_e|| / ||<sigma>||_F.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import spectral as sp
from .materials import isotropic_tensor, mandel_to_tensor4, sym_to_mandel, mandel_to_sym

SMALL = "small"
FINITE = "finite"


class IsoTangent:
    """Per-voxel isotropic stiffness, sigma = lam tr(eps) I + 2 mu eps."""

    def __init__(self, lam, mu):
        self.lam = np.asarray(lam, dtype=np.float64)
        self.mu = np.asarray(mu, dtype=np.float64)

    def stress(self, eps):
        tr = eps[0, 0] + eps[1, 1] + eps[2, 2]
        out = 2.0 * self.mu * eps
        for i in range(3):
            out[i, i] = out[i, i] + self.lam * tr
        return out

    def mean(self):
        return isotropic_tensor(float(np.mean(self.lam)), float(np.mean(self.mu)))


class GeneralTangent:
    """Per-voxel fourth-order tensor C[x, y, z, i, j, k, l]; sigma_ij = C_ijkl eps_kl.
    Also serves the finite-strain tangent K_iJkL acting on H_kL."""

    def __init__(self, C):
        self.C = np.asarray(C, dtype=np.float64)

    def stress(self, eps):
        return np.einsum("xyzijkl,klxyz->ijxyz", self.C, eps)

    def mean(self):
        return self.C.mean(axis=(0, 1, 2))


class Space:
    """Discrete setting of one RVE: grid, frequencies, null set, weights and
    the macroscopic basis restricted to the stress-controlled set S."""

    def __init__(self, shape, kin=SMALL, stress_mask=None, lengths=None):
        self.shape = tuple(int(v) for v in shape)
        self.N = float(np.prod(self.shape))
        self.kin = kin
        self.xi = sp.xi_half(self.shape, lengths)
        self.Z = sp.null_set(self.shape)
        self.w = sp.half_weights(self.shape)
        if stress_mask is None:
            stress_mask = np.zeros((3, 3), dtype=bool)
        self.mask = np.asarray(stress_mask, dtype=bool)
        if kin == SMALL:
            if not np.array_equal(self.mask, self.mask.T):
                raise ValueError("small strains need a symmetric stress mask")
            basis, pairs = sp.mandel_basis(), sp.MANDEL_PAIRS
        else:
            basis, pairs = sp.full_basis(), tuple((a // 3, a % 3) for a in range(9))
        self.basis = basis
        self.S = [a for a, (i, j) in enumerate(pairs) if self.mask[i, j]]
        self.BS = basis[self.S] if self.S else np.zeros((0, 3, 3))
        self.grad = sp.sym_grad if kin == SMALL else sp.full_grad

    # vectors are pairs (a, e)
    def zeros(self):
        return (np.zeros((3,) + sp.half_shape(self.shape), dtype=complex), np.zeros(len(self.S)))

    def dot(self, u, v):
        return sp.inner(u[0], v[0], self.w) + float(np.dot(u[1], v[1]))

    def macro_tensor(self, e):
        return np.einsum("a,aij->ij", e, self.BS)

    def macro_row(self, t):
        return np.einsum("aij,ij->a", self.BS, t)

    def field_of(self, a, e, E):
        """Real strain (or displacement-gradient) field E + e + grad(u)."""
        g = sp.real_field(self.grad(a, self.xi), self.shape)
        return g + (E + self.macro_tensor(e))[:, :, None, None, None]

    def divergence_residual(self, sig):
        """(i xi_j F[sigma]_ij / N, <sigma>) with the null set cleared."""
        s = sp.fourier(sig, self.shape)
        r = sp.div(s, self.xi)
        r[:, self.Z] = 0.0
        return r, s[:, :, 0, 0, 0].real.copy()

    def apply(self, x, tangent, E=None):
        """K{a|e} for a linear tangent; also returns <sigma> of the field."""
        if E is None:
            E = np.zeros((3, 3))
        eps = self.field_of(x[0], x[1], E)
        r, dc = self.divergence_residual(tangent.stress(eps))
        return (-r, self.macro_row(dc)), dc

    def preconditioner(self, Cbar):
        """Returns z = M r for M of eqs. pred2/pred3."""
        A = np.einsum("j...,ijkl,l...->...ik", self.xi, Cbar, self.xi)
        nz = ~self.Z
        Minv = np.zeros(A.shape)
        Minv[nz] = np.linalg.inv(A[nz])
        if self.S:
            Ce = np.einsum("aij,ijkl,bkl->ab", self.BS, Cbar, self.BS)
            Me = np.linalg.inv(Ce)
        else:
            Me = np.zeros((0, 0))

        def apply_m(r):
            za = np.einsum("...ik,k...->i...", Minv, r[0])
            return (za, Me @ r[1])
        return apply_m


def coarse_points(space, kc):
    """Half-spectrum points of the coarse Fourier set: every signed
    frequency |m_a| <= kc on all three axes, xi != 0, and on the
    self-conjugate planes one point of each pair (k, -k).  Returns a list
    of (k1, k2, k3)."""
    n1, n2, n3 = space.shape
    h3 = n3 // 2 + 1

    def sgn(k, n):
        return k if k <= n // 2 else k - n

    pts, seen = [], set()
    for k1 in range(n1):
        for k2 in range(n2):
            for k3 in range(h3):
                if max(abs(sgn(k1, n1)), abs(sgn(k2, n2)), abs(sgn(k3, n3))) > kc or space.Z[k1, k2, k3]:
                    continue
                plane = k3 == 0 or (n3 % 2 == 0 and k3 == n3 // 2)
                if plane:
                    kp = ((-k1) % n1, (-k2) % n2, k3)
                    if kp in seen:
                        continue
                    seen.add((k1, k2, k3))
                pts.append((k1, k2, k3))
    return pts


class TwoLevelPreconditioner:
    """Preconditioner with an exact coarse block (a two-level variant of
    Sec. 2.5 eqs. pred2/pred3).  M(xi) = [xi.Cbar.xi]^-1 is the inverse of
    the operator's per-frequency diagonal block for the homogeneous mean
    medium.  Here the unknowns on the coarse Fourier set (coarse_points)
    instead get the inverse of the heterogeneous operator's own block on
    that set, E = e_i . K e_j, with e_i the orthonormal real basis of the
    coarse unknowns (a unit or imaginary unit at one point and component,
    scaled by 1/sqrt(2), with its conjugate partner on the self-conjugate
    planes); every other frequency keeps M(xi), the macro block keeps
    [B:Cbar:B]^-1.  The result is block diagonal with SPD blocks, so SPD.
    E is built by applying K to every coarse basis vector (its definition)."""

    def __init__(self, space, tangent, kc):
        self.space = space
        self.M0 = space.preconditioner(tangent.mean())
        self.pts = coarse_points(space, kc)
        self.m = 6 * len(self.pts)
        cols = []
        for j in range(self.m):
            (q, _), _ = space.apply((self.basis(j), np.zeros(len(space.S))), tangent)
            cols.append(self.coords(q))
        E = np.array(cols).T
        self.E = 0.5 * (E + E.T)
        self.Einv = np.linalg.inv(self.E)

    def _unit(self, j):
        p, rest = divmod(j, 6)
        c, part = divmod(rest, 2)
        return self.pts[p], c, (1j if part else 1.0)

    def basis(self, j):
        """Coarse basis vector j (field part)."""
        space = self.space
        n1, n2, n3 = space.shape
        a = np.zeros((3,) + sp.half_shape(space.shape), dtype=complex)
        k, c, u = self._unit(j)
        a[(c,) + k] = u / np.sqrt(2.0)
        if k[2] == 0 or (n3 % 2 == 0 and k[2] == n3 // 2):
            kp = ((-k[0]) % n1, (-k[1]) % n2, k[2])
            a[(c,) + kp] = np.conj(u) / np.sqrt(2.0)
        return a

    def coords(self, a):
        """<e_j, a> for every coarse basis vector: sqrt(2) Re(conj(u) a(k))."""
        out = np.zeros(self.m)
        for j in range(self.m):
            k, c, u = self._unit(j)
            out[j] = np.sqrt(2.0) * float(np.real(np.conj(u) * a[(c,) + k]))
        return out

    def __call__(self, r):
        za, ze = self.M0(r)
        za = za.copy()
        y = self.Einv @ self.coords(r[0])
        n1, n2, n3 = self.space.shape
        for j in range(self.m):
            k, c, u = self._unit(j)
            za[(c,) + k] = 0.0
            if k[2] == 0 or (n3 % 2 == 0 and k[2] == n3 // 2):
                za[(c,) + ((-k[0]) % n1, (-k[1]) % n2, k[2])] = 0.0
        for j in range(self.m):
            za = za + y[j] * self.basis(j)
        return za, ze


@dataclass
class PCGInfo:
    iterations: int = 0
    converged: bool = False
    breakdown: bool = False
    eq_res: float = np.inf
    load_res: float = np.inf
    history: list = field(default_factory=list)


def residual_norms(space, r, sig, scale=None):
    """Equilibrium and loading residuals relative to ||<sigma>|| (Sec. 3),
    or to a fixed `scale` when one is given."""
    nrm = float(np.linalg.norm(sig)) if scale is None else float(scale)
    ra = np.sqrt(max(sp.inner(r[0], r[0], space.w), 0.0))
    re = float(np.linalg.norm(r[1]))
    if nrm == 0.0:
        return (0.0 if ra == 0.0 else np.inf), (0.0 if re == 0.0 else np.inf)
    return ra / nrm, re / nrm


def pcg(space, tangent, precond, b, sig0, tol=1e-8, tol_load=1e-10, max_iter=10000,
        x0=None, keep_history=False, scale=None):
    """Preconditioned conjugate gradient on K{a|e} = b (Sec. 3 intro: CG for
    complex numbers with the preconditioner of eqs. pred2/pred3).

    sig0 is <sigma> of the field that produced b; the average stress of the
    current iterate is tracked as sig0 + <sigma>(K x).  Stops when the
    equilibrium residual is below tol and the loading residual below
    tol_load (checked before the first iteration too).  `scale` replaces
    ||<sigma>|| in both tests when given."""
    info = PCGInfo()
    if x0 is None:
        x = space.zeros()
        r = (b[0].copy(), b[1].copy())
        sig = np.array(sig0, dtype=np.float64)
    else:
        x = (x0[0].copy(), x0[1].copy())
        Kx, dcx = space.apply(x, tangent)
        r = (b[0] - Kx[0], b[1] - Kx[1])
        sig = np.array(sig0, dtype=np.float64) + dcx
    z = precond(r)
    p = (z[0].copy(), z[1].copy())
    rz = space.dot(r, z)
    while True:
        eq, ld = residual_norms(space, r, sig, scale)
        info.eq_res, info.load_res = eq, ld
        if keep_history:
            info.history.append(eq)
        if eq < tol and ld < tol_load:
            info.converged = True
            break
        if info.iterations >= max_iter:
            break
        q, dcp = space.apply(p, tangent)
        pq = space.dot(p, q)
        if not pq > 0.0:
            info.breakdown = True
            break
        alpha = rz / pq
        x = (x[0] + alpha * p[0], x[1] + alpha * p[1])
        r = (r[0] - alpha * q[0], r[1] - alpha * q[1])
        sig = sig + alpha * dcp
        z = precond(r)
        rz_new = space.dot(r, z)
        beta = rz_new / rz
        rz = rz_new
        p = (z[0] + beta * p[0], z[1] + beta * p[1])
        info.iterations += 1
    return x, sig, info


@dataclass
class BlockPCGInfo:
    iterations: int = 0          # block iterations
    applies: int = 0             # operator applications (sum of the block widths)
    converged: bool = False
    breakdown: bool = False
    col_iterations: list = field(default_factory=list)  # block iteration at which each column stopped
    eq_res: list = field(default_factory=list)
    load_res: list = field(default_factory=list)


def _orthonormalize(space, W, drop_tol, ref=None):
    """Orthonormal basis (for space.dot) of the span of the vectors W:
    Cholesky factorization of their Gram matrix with diagonal pivoting,
    G[perm][:, perm] = L L^T over the kept columns, then P = W[perm] L^-T.
    The pivot of a column is the squared norm of its part orthogonal to the
    kept ones; the column is dropped as dependent when that is not above
    drop_tol times ref[j] (default: its own squared norm)."""
    m = len(W)
    if m == 0:
        return []
    G = np.array([[space.dot(W[i], W[k]) for k in range(m)] for i in range(m)])
    d = np.diag(G).astype(np.float64).copy()
    ref = d.copy() if ref is None else np.asarray(ref, dtype=np.float64)
    Lrow = np.zeros((m, m))  # Lrow[i, t]: entry of original column i in pivot step t
    perm, rest = [], list(range(m))
    for t in range(m):
        rest = [i for i in rest if d[i] > drop_tol * ref[i]]
        if not rest:
            break
        j = max(rest, key=lambda i: d[i])
        piv = np.sqrt(d[j])
        Lrow[j, t] = piv
        rest.remove(j)
        for i in rest:
            Lrow[i, t] = (G[i, j] - np.dot(Lrow[i, :t], Lrow[j, :t])) / piv
            d[i] -= Lrow[i, t] ** 2
        perm.append(j)
    k = len(perm)
    L = Lrow[perm, :k]                      # k x k lower triangular
    C = np.linalg.inv(L).T                  # L^-T
    return [(sum(C[u, t] * W[perm[u]][0] for u in range(k)), sum(C[u, t] * W[perm[u]][1] for u in range(k)))
            for t in range(k)]


def block_pcg(space, tangent, precond, B, sig0, tol=1e-8, tol_load=1e-10, max_iter=10000, drop_tol=1e-12):
    """Block preconditioned CG for s right-hand sides of one operator.

    The iterates of every column are taken from one block Krylov space of
    the preconditioned operator, spanned by the preconditioned residuals of
    all columns (the method of Sec. 3 -- CG for complex numbers with the
    preconditioner of eqs. pred2/pred3 -- with a block of directions in place
    of one).  With P a block of K-conjugate directions and Q = K P:
        alpha = (P^T Q)^-1 P^T R,   X += P alpha,   R -= Q alpha,
        beta  = -(P^T Q)^-1 Q^T Z (Z = M R),   next P: an orthonormal basis of Z + P beta,
    which keeps the new directions K-conjugate to the old ones.  A column
    whose residuals meet tol / tol_load (relative to its own ||<sigma>||, as
    in pcg) stops: its iterate and residual are no longer updated and its
    preconditioned residual leaves the block.  Dependent directions are
    dropped by the pivoted orthonormalization.

    B: list of s vectors (a, e); sig0: <sigma> of the fields that produced
    them (s, 3, 3).  Returns the iterates, the tracked <sigma> per column and
    a BlockPCGInfo."""
    s = len(B)
    info = BlockPCGInfo(col_iterations=[0] * s, eq_res=[np.inf] * s, load_res=[np.inf] * s)
    X = [space.zeros() for _ in range(s)]
    R = [(b[0].copy(), b[1].copy()) for b in B]
    sig = [np.array(v, dtype=np.float64) for v in sig0]

    def done(j):
        eq, ld = residual_norms(space, R[j], sig[j])
        info.eq_res[j], info.load_res[j] = eq, ld
        return eq < tol and ld < tol_load

    def comb(V, C, j):
        """sum_i V_i C[i, j]"""
        a = sum(C[i, j] * V[i][0] for i in range(len(V)))
        e = sum(C[i, j] * V[i][1] for i in range(len(V)))
        return a, e

    active = [j for j in range(s) if not done(j)]
    P = _orthonormalize(space, [precond(R[j]) for j in active], drop_tol) if active else []
    while active and P and info.iterations < max_iter:
        QD = [space.apply(p, tangent) for p in P]
        Q = [q for q, _ in QD]
        dcP = [dc for _, dc in QD]
        info.applies += len(P)
        m = len(P)
        Gam = np.array([[space.dot(P[i], Q[k]) for k in range(m)] for i in range(m)])
        Gam = 0.5 * (Gam + Gam.T)
        try:
            Lg = np.linalg.cholesky(Gam)
        except np.linalg.LinAlgError:
            info.breakdown = True
            break
        PR = np.array([[space.dot(P[i], R[j]) for j in active] for i in range(m)])
        alpha = np.linalg.solve(Lg.T, np.linalg.solve(Lg, PR))
        for jj, j in enumerate(active):
            da, de = comb(P, alpha, jj)
            qa, qe = comb(Q, alpha, jj)
            X[j] = (X[j][0] + da, X[j][1] + de)
            R[j] = (R[j][0] - qa, R[j][1] - qe)
            sig[j] = sig[j] + sum(alpha[i, jj] * dcP[i] for i in range(m))
        info.iterations += 1
        still = []
        for j in active:
            if done(j):
                info.col_iterations[j] = info.iterations
            else:
                still.append(j)
        active = still
        if not active:
            break
        Z = [precond(R[j]) for j in active]
        QZ = np.array([[space.dot(Q[i], Z[jj]) for jj in range(len(active))] for i in range(m)])
        beta = -np.linalg.solve(Lg.T, np.linalg.solve(Lg, QZ))
        W = []
        for jj in range(len(active)):
            pa, pe = comb(P, beta, jj)
            W.append((Z[jj][0] + pa, Z[jj][1] + pe))
        # a column of W that has lost nearly all of its preconditioned
        # residual to the conjugation brings no new direction
        P = _orthonormalize(space, W, drop_tol, [space.dot(z, z) for z in Z])
    for j in active:
        info.col_iterations[j] = info.iterations
    info.converged = not active
    return X, sig, info


def solve_linear_block(shape, tangent, loads, stress_mask=None, tol=1e-8, tol_load=1e-10, max_iter=10000,
                       kin=SMALL, coarse_kc=None):
    """The linear problems of several loads (one stress mask) solved by
    block_pcg; returns a LinearResult per load and the BlockPCGInfo."""
    space = Space(shape, kin, stress_mask)
    B, sig0, EUs = [], [], []
    for load in loads:
        E_U, sbar = split_load(space, load)
        (ka, _), dc0 = space.apply(space.zeros(), tangent, E_U)
        B.append((-ka, sbar - space.macro_row(dc0)))
        sig0.append(dc0)
        EUs.append(E_U)
    M = space.preconditioner(tangent.mean()) if coarse_kc is None else TwoLevelPreconditioner(space, tangent, coarse_kc)
    X, sig, info = block_pcg(space, tangent, M, B, sig0, tol, tol_load, max_iter)
    out = [LinearResult(x[0], x[1], sg, E_U + space.macro_tensor(x[1]), None, space, E_U)
           for x, sg, E_U in zip(X, sig, EUs)]
    return out, info


def split_load(space, load):
    """Prescribed strain part (zero on S) and the prescribed stress row."""
    load = np.asarray(load, dtype=np.float64)
    m = space.mask.astype(np.float64)
    return load * (1.0 - m), space.macro_row(load * m)


@dataclass
class LinearResult:
    a: np.ndarray
    e: np.ndarray
    sigma_bar: np.ndarray
    eps_bar: np.ndarray
    info: PCGInfo
    space: Space
    E_U: np.ndarray

    def strain_field(self):
        return self.space.field_of(self.a, self.e, self.E_U)


def solve_linear(shape, tangent, load, stress_mask=None, tol=1e-8, tol_load=1e-10,
                 max_iter=10000, x0=None, keep_history=False, kin=SMALL, coarse_kc=None, lengths=None):
    """Linear DBFFT solve (Sec. 2.2 strain control, Sec. 2.3 stress/mixed
    control): small-strain elasticity, or (kin=FINITE) the linearized
    finite-strain problem with a fixed tangent K (the system of one Newton
    step, Sec. 2.4).  `load` holds the prescribed strain (displacement
    gradient) on strain-controlled components and the prescribed stress on
    the components where stress_mask is true.  `lengths`: the cell's side
    lengths (Sec. 2.1), default 1, 1, 1."""
    space = Space(shape, kin, stress_mask, lengths)
    E_U, sbar = split_load(space, load)
    (ka, _), dc0 = space.apply(space.zeros(), tangent, E_U)
    b = (-ka, sbar - space.macro_row(dc0))
    M = space.preconditioner(tangent.mean()) if coarse_kc is None else TwoLevelPreconditioner(space, tangent, coarse_kc)
    x, sig, info = pcg(space, tangent, M, b, dc0, tol, tol_load, max_iter, x0, keep_history)
    eps_bar = E_U + space.macro_tensor(x[1])
    return LinearResult(x[0], x[1], sig, eps_bar, info, space, E_U)


def true_residual(space, tangent, res: LinearResult, load):
    """Equilibrium and loading residuals recomputed from the solution field."""
    eps = res.strain_field()
    r, dc = space.divergence_residual(tangent.stress(eps))
    _, sbar = split_load(space, load)
    return residual_norms(space, (r, sbar - space.macro_row(dc)), dc)


# ---------------------------------------------------------------------------
# Newton scheme (Sec. 2.4, eqs. lineariz, eqfinite, nonlineqf and
# nonlineqfstress).  Each Newton iteration linearizes the stress around the
# current field, solves the linear DBFFT system for {da | de} with the
# consistent tangent by PCG, and updates.  Stopping: the largest change of
# any component of the strain (small) or deformation gradient (finite) at
# any voxel during the last update is below newton_tol (Sec. 2.4).
# ---------------------------------------------------------------------------

@dataclass
class NewtonInfo:
    increments: int = 0
    newton_iters: list = field(default_factory=list)
    pcg_iters: list = field(default_factory=list)
    eq_res: list = field(default_factory=list)
    converged: bool = True
    sigma_bar: list = field(default_factory=list)
    eps_bar: list = field(default_factory=list)


def newton(shape, law, loads, stress_mask, kin=SMALL, tol=1e-8, tol_load=1e-10,
           newton_tol=1e-6, max_newton=25, max_iter=10000, refresh="increment",
           state=None, checkpoints=None, lengths=None):
    """Incremental Newton-DBFFT driver.

    law.update(field, state) -> (stress, tangent_obj, new_state) where field
    is the real strain (small) or displacement gradient H = F - I (finite)
    with layout (3, 3, n1, n2, n3).  loads: list of 3x3 prescribed values per
    increment (strain / F - I on strain-controlled components, stress on S).
    refresh: 'increment' recomputes the preconditioner's mean tangent at the
    first Newton iteration of every increment (Sec. 2.5), 'initial' only once.
    checkpoints: a list that receives, per increment, the converged (a, e,
    E_U) and the law state the increment started from.
    Returns (a, e, state, info)."""
    space = Space(shape, kin, stress_mask, lengths)
    a, e = space.zeros()
    info = NewtonInfo()
    Cbar = None
    for k, L in enumerate(loads):
        E_U, sbar = split_load(space, L)
        fld = space.field_of(a, e, E_U)
        its, pits = 0, 0
        conv = False
        for i in range(max_newton + 1):
            sig, tan, new_state = law.update(fld, state)
            if Cbar is None or (i == 0 and refresh == "increment"):
                Cbar = tan.mean()
            r_a, dc = space.divergence_residual(sig)
            r = (r_a, sbar - space.macro_row(dc))
            if i > 0 and dmax < newton_tol:
                conv = True
                break
            if i == max_newton:
                break
            M = space.preconditioner(Cbar)
            d, _, pinfo = pcg(space, tan, M, r, dc, tol, tol_load, max_iter)
            pits += pinfo.iterations
            if pinfo.breakdown or not pinfo.converged:
                break
            a = a + d[0]
            e = e + d[1]
            new_fld = space.field_of(a, e, E_U)
            dmax = float(np.max(np.abs(new_fld - fld)))
            fld = new_fld
            its += 1
        eq, _ = residual_norms(space, r, dc)
        if checkpoints is not None:
            checkpoints.append((a.copy(), e.copy(), E_U.copy(), state))
        state = new_state
        info.increments += 1
        info.newton_iters.append(its)
        info.pcg_iters.append(pits)
        info.eq_res.append(eq)
        info.converged = info.converged and conv
        info.sigma_bar.append(dc.copy())
        avg = E_U + space.macro_tensor(e)
        info.eps_bar.append(avg)
    return a, e, state, info


class J2Law:
    """Small-strain law object for newton(): rate-dependent J2 with per-voxel
    Mandel elastic stiffness C (n1, n2, n3, 6, 6)."""

    def __init__(self, C_mandel, s0, m, edot0, dt):
        """s0 is a scalar or one flow stress per voxel (n1, n2, n3)."""
        self.C = np.asarray(C_mandel, dtype=np.float64)
        self.s0, self.m, self.edot0, self.dt = s0, m, edot0, dt
        self.shape = self.C.shape[:3]

    def initial_state(self):
        return np.zeros(self.shape + (6,))

    def update(self, eps, state):
        from .materials import j2vp_return_map
        if state is None:
            state = self.initial_state()
        nv = int(np.prod(self.shape))
        ev = np.moveaxis(sym_to_mandel(eps), 0, -1).reshape(nv, 6)
        s0 = np.broadcast_to(np.asarray(self.s0, dtype=np.float64), self.shape).reshape(nv)
        sig, dp, ep, tan = j2vp_return_map(ev, state.reshape(nv, 6), self.C.reshape(nv, 6, 6),
                                           s0, self.m, self.edot0, self.dt)
        sig_t = mandel_to_sym(np.moveaxis(sig.reshape(self.shape + (6,)), -1, 0))
        Ct = mandel_to_tensor4(tan.reshape(self.shape + (6, 6)))
        return sig_t, GeneralTangent(Ct), ep.reshape(self.shape + (6,))


class SVKLaw:
    """Saint Venant-Kirchhoff law object for newton() (Sec. 3.3): field is
    H = F - I."""

    def __init__(self, mu, lam):
        self.mu = np.asarray(mu, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)

    def update(self, H, state):
        from .materials import svk_stress, svk_tangent
        F = np.moveaxis(H, (0, 1), (-2, -1)) + np.eye(3)
        P = svk_stress(F, self.mu, self.lam)
        K = svk_tangent(F, self.mu, self.lam)
        return np.moveaxis(P, (-2, -1), (0, 1)), GeneralTangent(K), state


class NeoHookeLaw:
    """Finite-strain law object for newton(): field is H = F - I."""

    def __init__(self, mu, lam):
        self.mu = np.asarray(mu, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)

    def update(self, H, state):
        from .materials import neohooke_stress, neohooke_tangent
        F = np.moveaxis(H, (0, 1), (-2, -1)) + np.eye(3)
        P = neohooke_stress(F, self.mu, self.lam)
        K = neohooke_tangent(F, self.mu, self.lam)
        return np.moveaxis(P, (-2, -1), (0, 1)), GeneralTangent(K), state


# ---------------------------------------------------------------------------
# Adjoint gradient of a homogenized response with respect to per-voxel
# moduli (not in the paper).  For J = G:<sigma> + H:<eps> at the solution of
# the linear problem, the Lagrangian gives dJ/dtheta(x) = (1/N) eta:dC/dtheta:eps
# where eta solves the same DBFFT system with prescribed strain G on the
# strain-controlled set and prescribed stress -H on S.
# ---------------------------------------------------------------------------

def adjoint_gradient_hyperelastic(shape, law, loads, stress_mask, G, H, tol=1e-12, newton_tol=1e-12):
    """Hyperelastic finite-strain counterpart (not in the paper): J = G:<P> +
    H:<F> at the end of the load path `loads` (as for newton()), and its
    gradient with respect to a per-voxel factor theta(x) on the law's moduli
    at theta = 1.  The end state does not depend on the path, so with the
    tangent K of the final state the Lagrangian gives: eta solves the
    linearized cell problem with prescribed gradient G on the controlled
    components and stress -H on S, and dJ/dtheta(x) = (G + grad eta):dP/dtheta
    / N with dP/dtheta = P (P linear in the moduli).
    Returns (J, gradient field, newton info)."""
    a, e, state, info = newton(shape, law, loads, stress_mask, kin=FINITE, tol=tol, tol_load=tol,
                               newton_tol=newton_tol)
    space = Space(shape, FINITE, stress_mask)
    E_U, _ = split_load(space, loads[-1])
    Hf = space.field_of(a, e, E_U)
    P, K, _ = law.update(Hf, state)
    mask = np.asarray(stress_mask if stress_mask is not None else np.zeros((3, 3)), bool)
    G = np.asarray(G, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    adj = solve_linear(shape, K, np.where(mask, -H, G), stress_mask, tol, tol, kin=FINITE)
    Hadj = adj.strain_field()
    N = float(np.prod(shape))
    g = np.einsum("ij...,ij...->...", Hadj, P) / N
    J = float(np.sum(G * info.sigma_bar[-1]) + np.sum(H * (info.eps_bar[-1] + np.eye(3))))
    return J, g, info


def adjoint_gradient_j2(shape, law, loads, stress_mask, G, H, tol=1e-12, newton_tol=1e-12, max_iter=10000):
    """J2 viscoplastic counterpart (not in the paper): J = G:<sigma> + H:<eps>
    after the increments `loads` (as for newton(); the response depends on
    the path), and its gradient with respect to a per-voxel factor theta(x)
    on the flow stress s0 at theta = 1.

    Per voxel and increment n the return map gives sigma_n from eps_n -
    p_{n-1} (p the plastic strain, Mandel vectors) with the consistent
    tangent K_n, and p_n = eps_n - S sigma_n (S the elastic compliance);
    the flow increment dp_n scales as -m dp_n with theta.  Going back from
    the last increment with lambda (the multiplier of p_n, zero after the
    last increment):
      A_n    = lambda - K_n S lambda                         (prestress)
      eps*_n = adjoint field of the linearized cell problem with tangent K_n,
               stress law K_n:eps + A_n, prescribed strain G on the
               controlled components and stress -H on S at the last
               increment, zero at the others (PCG stopped on the residual
               relative to its initial value)
      lambda <- K_n (S lambda - eps*_n)
      grad  += -(m / N) dp_n . lambda
    Returns (J, gradient field, newton info)."""
    ck = []
    a, e, state, info = newton(shape, law, loads, stress_mask, kin=SMALL, tol=tol, tol_load=tol,
                               newton_tol=newton_tol, max_iter=max_iter, checkpoints=ck)
    from .materials import j2vp_return_map
    space = Space(shape, SMALL, stress_mask)
    nv = int(np.prod(shape))
    C = law.C.reshape(nv, 6, 6)
    Sc = np.linalg.inv(C)
    s0 = np.broadcast_to(np.asarray(law.s0, dtype=np.float64), shape).reshape(nv)
    mask = np.asarray(stress_mask if stress_mask is not None else np.zeros((3, 3)), bool)
    G = np.asarray(G, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    lam = np.zeros((nv, 6))
    g = np.zeros(nv)
    for n in reversed(range(len(loads))):
        an, en, EUn, p_prev = ck[n]
        p_prev = (law.initial_state() if p_prev is None else p_prev).reshape(nv, 6)
        eps = space.field_of(an, en, EUn)
        ev = np.moveaxis(sym_to_mandel(eps), 0, -1).reshape(nv, 6)
        _, _, p_n, K = j2vp_return_map(ev, p_prev, C, s0, law.m, law.edot0, law.dt)
        dp = p_n - p_prev
        KSlam = np.einsum("vab,vb->va", K, np.einsum("vab,vb->va", Sc, lam))
        A = lam - KSlam
        load = np.where(mask, -H, G) if n == len(loads) - 1 else np.zeros((3, 3))
        E_U, sbar = split_load(space, load)
        tan = GeneralTangent(mandel_to_tensor4(K.reshape(tuple(shape) + (6, 6))))
        sig0 = tan.stress(np.broadcast_to(E_U[:, :, None, None, None], (3, 3) + tuple(shape)))
        sig0 = sig0 + mandel_to_sym(np.moveaxis(A.reshape(tuple(shape) + (6,)), -1, 0))
        r_a, dc = space.divergence_residual(sig0)
        r = (r_a, sbar - space.macro_row(dc))
        # residual test relative to the initial residual: the mean stress of
        # these problems changes sign along the path
        scale = np.sqrt(max(sp.inner(r[0], r[0], space.w), 0.0) + float(np.sum(r[1] ** 2)))
        if scale > 0.0:
            d, _, pinfo = pcg(space, tan, space.preconditioner(tan.mean()), r, dc, tol, tol, max_iter, scale=scale)
            if not pinfo.converged:
                raise RuntimeError("adjoint solve did not converge")
        else:
            d = space.zeros()
        es = np.moveaxis(sym_to_mandel(space.field_of(d[0], d[1], E_U)), 0, -1).reshape(nv, 6)
        lam = KSlam - np.einsum("vab,vb->va", K, es)
        g += -(law.m / nv) * np.sum(dp * lam, axis=1)
    J = float(np.sum(G * info.sigma_bar[-1]) + np.sum(H * info.eps_bar[-1]))
    return J, g.reshape(shape), info


def adjoint_gradient(shape, tangent, dtangent, load, stress_mask, G, H, tol=1e-12,
                     max_iter=10000):
    """Returns (J, dJ/dtheta field (n1, n2, n3), forward result, adjoint result).
    dtangent: IsoTangent of dC/dtheta per voxel (e.g. C(E=1, nu))."""
    fwd = solve_linear(shape, tangent, load, stress_mask, tol, tol, max_iter)
    mask = np.asarray(stress_mask if stress_mask is not None else np.zeros((3, 3)), bool)
    G = np.asarray(G, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    adj_load = np.where(mask, -H, G)
    adj = solve_linear(shape, tangent, adj_load, stress_mask, tol, tol, max_iter)
    eps = fwd.strain_field()
    eta = adj.strain_field()
    N = float(np.prod(shape))
    g = np.einsum("ij...,ij...->...", eta, dtangent.stress(eps)) / N
    J = float(np.sum(G * fwd.sigma_bar) + np.sum(H * fwd.eps_bar))
    return J, g, fwd, adj
