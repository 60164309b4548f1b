"""Independent matrix formulation of the restricted iteration and the energies.

Test-only checker for the oracle.  Operators are built as explicit matrices
(Kronecker products of 1-D forward differences), the divergence is defined as
the negative transpose of the gradient matrix, and the restriction is a
diagonal mask, so none of the oracle's loop code is reused.
Paper: Sec. 2.1 (eq. DF and the alternating steps), Sec. 3 (restricted systems).
"""
import numpy as np


def diff_matrix(n):
    """1-D forward difference, last row zero (n x n)."""
    D = np.zeros((n, n))
    for i in range(n - 1):
        D[i, i] = -1.0
        D[i, i + 1] = 1.0
    return D


def grad_matrix(H, W):
    """G = [Dx; Dy] acting on row-major vectors of length H*W."""
    Dx = np.kron(np.eye(H), diff_matrix(W))
    Dy = np.kron(diff_matrix(H), np.eye(W))
    return np.vstack([Dx, Dy])


class Twin:
    def __init__(self, f, lam, theta, tau, delta):
        f = np.asarray(f, np.float32).astype(np.float64)
        self.H, self.W = f.shape
        self.N = f.size
        self.f = f.ravel()
        self.lam, self.theta, self.tau = lam, theta, tau
        self.A = np.abs(self.f) < delta
        self.h = (self.f < 0).astype(np.float64)
        self.G = grad_matrix(self.H, self.W)
        self.Div = -self.G.T

    def init(self, u0=None, p0=None):
        A, h = self.A, self.h
        u = h.copy()
        if u0 is not None:
            u[A] = np.asarray(u0, np.float64).ravel()[A]
        v = h.copy()
        v[A] = np.clip(u[A] - self.theta * self.lam * self.f[A], 0.0, 1.0)
        p = np.zeros(2 * self.N)
        if p0 is not None:
            q = np.concatenate([np.asarray(p0[0], np.float64).ravel(),
                                np.asarray(p0[1], np.float64).ravel()])
            col = np.tile(np.arange(self.W), self.H)
            row = np.repeat(np.arange(self.H), self.W)
            keep = np.concatenate([A & (col < self.W - 1), A & (row < self.H - 1)])
            p[keep] = q[keep]
        return u, v, p

    def step(self, u, v, p, inner=1):
        N, A, th, tau = self.N, self.A, self.theta, self.tau
        for _ in range(inner):
            d = self.Div @ p
            w = np.where(A, d, 0.0) - v / th      # v = H(-f) off the domain
            g = self.G @ w
            n = np.sqrt(g[:N] ** 2 + g[N:] ** 2)
            scale = 1.0 / (1.0 + tau * np.concatenate([n, n]))
            p = np.where(np.concatenate([A, A]), (p + tau * g) * scale, 0.0)
        d = self.Div @ p
        u = np.where(A, v - th * d, u)
        v = np.where(A, np.clip(u - th * self.lam * self.f, 0.0, 1.0), v)
        return u, v, p

    def run(self, iters, u0=None, p0=None, inner=1):
        u, v, p = self.init(u0, p0)
        for _ in range(iters):
            u, v, p = self.step(u, v, p, inner)
        H, W, N = self.H, self.W, self.N
        return u.reshape(H, W), v.reshape(H, W), np.stack([p[:N].reshape(H, W), p[N:].reshape(H, W)])


def restricted_energy(f, lam, theta, delta, u, v):
    """E_RD(u, v) = sum_{x in RD} |grad u(x)| + 1/(2 theta) sum_RD (u-v)^2 + lam sum_RD f v,
    with u = H(-f) off RD (Sec. 2.1 eq. DF restricted as in Sec. 3)."""
    f = np.asarray(f, np.float32).astype(np.float64)
    A = np.abs(f) < delta
    h = (f < 0).astype(np.float64)
    ub = np.where(A, u, h)
    G = grad_matrix(*f.shape)
    g = G @ ub.ravel()
    N = f.size
    tv = np.sqrt(g[:N] ** 2 + g[N:] ** 2)[A.ravel()].sum()
    return tv + ((u - v) ** 2)[A].sum() / (2 * theta) + lam * (f * v)[A].sum()


def dual_value(f, lam, theta, delta, p):
    """Dual of the restricted split energy for |p| <= 1 on RD, p = 0 off RD:
    D(p) = sum_{off RD} H(-f) div p + sum_RD [ -theta/2 (div p)^2 + min(0, div p + lam f) ]."""
    f = np.asarray(f, np.float32).astype(np.float64)
    A = np.abs(f) < delta
    h = (f < 0).astype(np.float64)
    G = grad_matrix(*f.shape)
    d = (-G.T @ np.concatenate([p[0].ravel(), p[1].ravel()])).reshape(f.shape)
    return (h * d)[~A].sum() + (-theta * d ** 2 / 2 + np.minimum(0.0, d + lam * f))[A].sum()


def rof_dual_objective(f, theta, delta, v, p):
    """Objective minimised by the restricted Chambolle step for fixed v:
    sum_RD (theta div p - v)^2 - 2 theta sum_{off RD} H(-f) div p."""
    f = np.asarray(f, np.float32).astype(np.float64)
    A = np.abs(f) < delta
    h = (f < 0).astype(np.float64)
    G = grad_matrix(*f.shape)
    d = (-G.T @ np.concatenate([p[0].ravel(), p[1].ravel()])).reshape(f.shape)
    return ((theta * d - v) ** 2)[A].sum() - 2 * theta * (h * d)[~A].sum()


def _shift(a, dy, dx):
    """b[y, x] = a[y + dy, x + dx], zero outside the grid."""
    H, W = a.shape
    out = np.zeros_like(a)
    ys_dst = slice(max(0, -dy), H - max(0, dy))
    xs_dst = slice(max(0, -dx), W - max(0, dx))
    ys_src = slice(max(0, dy), H - max(0, -dy))
    xs_src = slice(max(0, dx), W - max(0, -dx))
    out[ys_dst, xs_dst] = a[ys_src, xs_src]
    return out


def reverse_with_w_noise(f, lam, theta, tau, delta, iters, ubar, rng=None, amp=0.0):
    """FP64 reverse mode of the restricted iteration (default start) in which the
    forward dual argument w is perturbed by amp * (|div p| + |v/theta|) * N(0,1)
    at every step -- a model of rounding w in a lower precision.  With amp = 0
    it is a second, array-level formulation of the oracle's reverse sweep.
    Returns (fbar, lambar)."""
    f64 = np.asarray(f, np.float32).astype(np.float64)
    H, W = f64.shape
    A = np.abs(f64) < delta
    h = (f64 < 0).astype(np.float64)
    c = np.where(A, theta * lam * f64, 0.0)
    lastc = np.zeros((H, W), bool)
    lastc[:, -1] = True
    lastr = np.zeros((H, W), bool)
    lastr[-1, :] = True

    def div(px, py):
        return (px - _shift(px, 0, -1)) + (py - _shift(py, -1, 0))

    def fwd(px, py, v, nz):
        d = div(px, py)
        w = np.where(A, d, 0.0) - v / theta + nz * (np.abs(d) + np.abs(v / theta))
        gx = np.where(lastc, 0.0, _shift(w, 0, 1) - w)
        gy = np.where(lastr, 0.0, _shift(w, 1, 0) - w)
        m = 1.0 / (1.0 + tau * np.sqrt(gx ** 2 + gy ** 2))
        nx = np.where(A, (px + tau * gx) * m, 0.0)
        ny = np.where(A, (py + tau * gy) * m, 0.0)
        s = v - theta * div(nx, ny) - c
        return nx, ny, np.where(A, np.clip(s, 0.0, 1.0), h), gx, gy, m, s

    v = np.where(A, np.clip(h - c, 0.0, 1.0), h)
    states = [(np.zeros((H, W)), np.zeros((H, W)), v)]
    noises = []
    for _ in range(iters):
        nz = amp * rng.normal(size=(H, W)) if amp > 0 else 0.0
        noises.append(nz)
        nx, ny, vn, _, _, _, _ = fwd(*states[-1], nz)
        states.append((nx, ny, vn))
    pbx, pby, vb = np.zeros((H, W)), np.zeros((H, W)), np.zeros((H, W))
    S = np.zeros((H, W))
    for k in range(iters, 0, -1):
        nx, ny, _, gx, gy, m, s = fwd(*states[k - 1], noises[k - 1])
        sb = np.where(A & (s > 0) & (s < 1), vb, 0.0)
        ub = np.where(A, sb + (ubar if k == iters else 0.0), 0.0)
        S += sb
        ptx = np.where(A, pbx + theta * np.where(lastc, 0.0, _shift(ub, 0, 1) - ub), 0.0)
        pty = np.where(A, pby + theta * np.where(lastr, 0.0, _shift(ub, 1, 0) - ub), 0.0)
        n = np.sqrt(gx ** 2 + gy ** 2)
        inv_n = np.where(n > 0, 1.0 / np.where(n > 0, n, 1.0), 0.0)
        k2 = tau * m * (nx * ptx + ny * pty) * inv_n
        gbx = np.where(A & ~lastc, tau * m * ptx - k2 * gx, 0.0)
        gby = np.where(A & ~lastr, tau * m * pty - k2 * gy, 0.0)
        wb = np.where(A, -div(gbx, gby), 0.0)
        pbx = np.where(A & ~lastc, m * ptx - np.where(lastc, 0.0, _shift(wb, 0, 1) - wb), 0.0)
        pby = np.where(A & ~lastr, m * pty - np.where(lastr, 0.0, _shift(wb, 1, 0) - wb), 0.0)
        vb = np.where(A, ub - wb / theta, 0.0)
    return np.where(A, -theta * lam * S, 0.0), float((-theta * f64 * S)[A].sum())



def dense_primal_dual_split(f, lam, theta, delta, t=0.025, tol=1e-15, max_iters=400000):
    """Brute-force dense solve of the restricted split energy (Sec. 2.1 eq. DF,
    restricted as in Sec. 3) by projected primal-dual gradient steps on its
    saddle form
        min over (u, v), 0 <= v <= 1 on RD,  max over |p(x)| <= 1 on RD, of
        <G u~, p> + |u - v|^2_RD / (2 theta) + lam <f, v>_RD,
    u~ = u on RD and H(-f) elsewhere, p = 0 off RD.  This is the first-order
    primal-dual method of Chambolle and Pock (steps t, s with t s |G|^2 < 1,
    |G|^2 <= 8) with the exact per-pixel proximal map of the (u, v) part: a
    different algorithm from the alternation that the paper iterates, with its
    own dense operator.  It runs until no coordinate moves by more than tol in
    one step, then as many steps again (the tail is linear, so the second half
    takes the error to rounding level).  Returns (u, v, steps)."""
    f = np.asarray(f, np.float32).astype(np.float64)
    H, W = f.shape
    N = f.size
    fv = f.ravel()
    A = np.abs(fv) < delta
    h = (fv < 0).astype(np.float64)
    G = grad_matrix(H, W)
    AA = np.concatenate([A, A])
    s = 0.999 / (8.0 * t)
    u, v = h.copy(), h.copy()
    ub = u.copy()
    p = np.zeros(2 * N)
    stop = max_iters
    k = 0
    while k < stop:
        q = p + s * (G @ ub)
        n = np.sqrt(q[:N] ** 2 + q[N:] ** 2)
        q = q / np.maximum(1.0, np.concatenate([n, n]))
        p = np.where(AA, q, 0.0)
        a = u - t * (G.T @ p)
        # argmin over v in [0,1], u of (|u-a|^2 + |v-v_k|^2)/(2t) + (u-v)^2/(2 theta) + lam f v:
        # u = (theta a + t v) / (theta + t) for each v, leaving a 1-D quadratic in v
        vn = (a / (theta + t) + v / t - lam * fv) / (1.0 / (theta + t) + 1.0 / t)
        vn = np.where(A, np.clip(vn, 0.0, 1.0), h)
        un = np.where(A, (theta * a + t * vn) / (theta + t), h)
        r = max(np.abs(un - u).max(), np.abs(vn - v).max())
        ub = 2.0 * un - u
        u, v = un, vn
        k += 1
        if stop == max_iters and k > 10 and r < tol:
            stop = min(max_iters, 2 * k)
    if stop == max_iters:
        raise RuntimeError("dense primal-dual solve did not reach its tolerance")
    return u.reshape(H, W), v.reshape(H, W), k


def pd_twin(f, lam, tau, sigma, delta, iters):
    """Restricted first-order primal-dual iteration for eq. CR (Sec. 5 carries
    the restriction of Sec. 3 over to other solvers), written from Chambolle
    and Pock's algorithm with extrapolation parameter 1 and dense operators:
        p    <- projection onto |p(x)| <= 1 of p + sigma G ubar   (RD rows)
        u'   <- clamp(u - tau (G^T p + lam f), 0, 1)              (RD)
        ubar <- 2 u' - u
    with u = ubar = H(-f) and p = 0 off RD.  Returns (u, p) after `iters`."""
    f = np.asarray(f, np.float32).astype(np.float64)
    H, W = f.shape
    N = f.size
    fv = f.ravel()
    A = np.abs(fv) < delta
    h = (fv < 0).astype(np.float64)
    G = grad_matrix(H, W)
    AA = np.concatenate([A, A])
    u = h.copy()
    ub = u.copy()
    p = np.zeros(2 * N)
    for _ in range(iters):
        q = p + sigma * (G @ ub)
        n = np.sqrt(q[:N] ** 2 + q[N:] ** 2)
        q = q / np.maximum(1.0, np.concatenate([n, n]))
        p = np.where(AA, q, 0.0)
        un = np.where(A, np.clip(u - tau * (G.T @ p + lam * fv), 0.0, 1.0), h)
        ub = 2.0 * un - u
        u = un
    return u.reshape(H, W), p.reshape(2, H, W)
