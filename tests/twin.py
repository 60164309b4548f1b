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
