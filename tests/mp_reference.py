"""Arbitrary-precision brute-force reference for tiny lattices (test code).

Independent of both the oracle and the GPU library.  Every step of the
method is done the most direct way available in mpmath:

* shells: roots of L_Np found with mpmath's polynomial root finder;
* truncated equilibrium: the least-squares projection of f_eq / omega onto
  the light-cone polynomials of degree <= N in the e^{-p} inner product
  (Sec. 2.2), built from numerically integrated moments (analytic radial
  integral, periodic trapezoid rule in angle, which converges geometrically
  for these smooth integrands) and normal equations solved by mpmath;
* Landau frame: mpmath's eigen-solver on T^mu_nu, largest real eigenvalue.
"""
import mpmath as mp


def laguerre_coeffs(n):
    """Power-series coefficients (low to high) of L_n."""
    return [mp.mpf((-1) ** k) * mp.binomial(n, k) / mp.factorial(k) for k in range(n + 1)]


def quadrature(Np, K, rotate=True):
    c = laguerre_coeffs(Np)
    roots = sorted([mp.re(r) for r in mp.polyroots(list(reversed(c)), maxsteps=200, extraprec=200)])
    cn = laguerre_coeffs(Np + 1)
    vel = []
    for i, pi_ in enumerate(roots):
        L = mp.polyval(list(reversed(cn)), pi_)
        wr = pi_ / ((Np + 1) ** 2 * L ** 2)
        for j in range(K):
            th = (j + (mp.mpf(i) / Np if rotate else 0)) * 2 * mp.pi / K
            vel.append((pi_, mp.cos(th), mp.sin(th), wr * 2 * mp.pi / K))
    return vel


def monomials(N):
    out = []
    for d in range(N + 1):
        for a in range(min(1, d) + 1):
            for b in range(d - a, -1, -1):
                out.append((a, b, d - a - b))
    return out


def _gram(N):
    mons = monomials(N)

    def ang(b, c):
        if b % 2 or c % 2:
            return mp.mpf(0)
        return 2 * mp.gamma(mp.mpf(b + 1) / 2) * mp.gamma(mp.mpf(c + 1) / 2) / mp.gamma(mp.mpf(b + c) / 2 + 1)

    G = mp.matrix(len(mons), len(mons))
    for r, (a1, b1, c1) in enumerate(mons):
        for s, (a2, b2, c2) in enumerate(mons):
            G[r, s] = mp.factorial(a1 + b1 + c1 + a2 + b2 + c2) * ang(b1 + b2, c1 + c2)
    return mons, G


def feq_moments_numeric(mons, n, T, U, M=128):
    """int f_eq m(p) dtheta dp for each monomial, f_eq = n/(2 pi T^2) e^{-U.p/T}."""
    out = []
    for (a, b, c) in mons:
        k = a + b + c
        acc = mp.mpf(0)
        for t in range(M):
            th = 2 * mp.pi * t / M
            ct, st = mp.cos(th), mp.sin(th)
            A = U[0] - U[1] * ct - U[2] * st
            acc += ct ** b * st ** c * mp.factorial(k) * (T / A) ** (k + 1)
        out.append(n / (2 * mp.pi * T ** 2) * acc * 2 * mp.pi / M)
    return out


class Lattice:
    """bc = (bc_x, bc_y), each 'periodic', 'wall' (a source across the edge
    is replaced by the target cell's population of the opposite velocity) or
    'fixed' (a source across the edge keeps the initial population of the
    nearest cell)."""

    def __init__(self, Np, K, N, nx, ny, fields, tau, dt, dps=40, bc=("periodic", "periodic")):
        mp.mp.dps = dps
        self.bc = bc
        self.vel = quadrature(Np, K)
        # opposite velocity: same shell, (cos, sin) -> (-cos, -sin), found by search
        self.opp = []
        for (p, ct, st, w) in self.vel:
            self.opp.append(min(range(len(self.vel)), key=lambda u: abs(self.vel[u][0] - p)
                                + abs(self.vel[u][1] + ct) + abs(self.vel[u][2] + st)))
        self.mons, self.G = _gram(N)
        self.nx, self.ny, self.tau, self.dt = nx, ny, mp.mpf(tau), mp.mpf(dt)
        n, T, ux, uy = fields
        self.f = {}
        for y in range(ny):
            for x in range(nx):
                U = self._U(mp.mpf(ux[y][x]), mp.mpf(uy[y][x]))
                fe = self.feq(mp.mpf(n[y][x]), mp.mpf(T[y][x]), U)
                for v in range(len(self.vel)):
                    self.f[(v, y, x)] = fe[v]
        self.f0 = dict(self.f)

    def _source(self, v, y, x, ys, xs):
        """Population of velocity v at the upwind point (xs, ys) of target (x, y)."""
        outside = []
        for axis, (i, n) in enumerate(((xs, self.nx), (ys, self.ny))):
            if self.bc[axis] == "periodic":
                continue
            if not 0 <= i < n:
                outside.append(self.bc[axis])
        xs, ys = xs % self.nx if self.bc[0] == "periodic" else xs, ys % self.ny if self.bc[1] == "periodic" else ys
        if "wall" in outside:
            return self.f[(self.opp[v], y, x)]
        if outside:
            return self.f0[(v, min(max(ys, 0), self.ny - 1), min(max(xs, 0), self.nx - 1))]
        return self.f[(v, ys, xs)]

    @staticmethod
    def _U(ux, uy):
        return (mp.sqrt(1 + ux * ux + uy * uy), ux, uy)

    def feq(self, n, T, U):
        mu = feq_moments_numeric(self.mons, n, T, U)
        coef = mp.lu_solve(self.G, mp.matrix(mu))
        out = []
        for (p, ct, st, w) in self.vel:
            val = mp.mpf(0)
            for s, (a, b, c) in enumerate(self.mons):
                val += coef[s] * p ** a * (p * ct) ** b * (p * st) ** c
            out.append(w * val)
        return out

    def moments(self, fs):
        m = [mp.mpf(0)] * 9
        for v, (p, ct, st, w) in enumerate(self.vel):
            P = (p, p * ct, p * st)
            fv = fs[v]
            m[0] += P[0] * fv; m[1] += P[1] * fv; m[2] += P[2] * fv
            m[3] += P[0] * P[0] * fv; m[4] += P[0] * P[1] * fv; m[5] += P[0] * P[2] * fv
            m[6] += P[1] * P[1] * fv; m[7] += P[1] * P[2] * fv; m[8] += P[2] * P[2] * fv
        return m

    @staticmethod
    def landau(m):
        Tm = mp.matrix([[m[3], m[4], m[5]], [m[4], m[6], m[7]], [m[5], m[7], m[8]]])
        eta = mp.diag([1, -1, -1])
        E, V = mp.eig(Tm * eta)
        k = max(range(3), key=lambda i: mp.re(E[i]))
        eps = mp.re(E[k])
        U = [mp.re(V[i, k]) for i in range(3)]
        nrm = mp.sqrt(U[0] ** 2 - U[1] ** 2 - U[2] ** 2)
        if U[0] < 0:
            nrm = -nrm
        U = [u / nrm for u in U]
        n = U[0] * m[0] - U[1] * m[1] - U[2] * m[2]
        return n, eps, U

    def step(self):
        nx, ny = self.nx, self.ny
        fs = {}
        for v, (p, ct, st, w) in enumerate(self.vel):
            ax, ay = self.dt * abs(ct), self.dt * abs(st)
            sx = 1 if ct >= 0 else -1
            sy = 1 if st >= 0 else -1
            for y in range(ny):
                for x in range(nx):
                    src = lambda ys, xs: self._source(v, y, x, ys, xs)
                    fs[(v, y, x)] = ((1 - ax) * (1 - ay) * self.f[(v, y, x)] + ax * (1 - ay) * src(y, x - sx)
                                     + (1 - ax) * ay * src(y - sy, x) + ax * ay * src(y - sy, x - sx))
        nv = len(self.vel)
        for y in range(ny):
            for x in range(nx):
                loc = [fs[(v, y, x)] for v in range(nv)]
                n, eps, U = self.landau(self.moments(loc))
                T = eps / (2 * n)
                fe = self.feq(n, T, U)
                for v, (p, ct, st, w) in enumerate(self.vel):
                    om = self.dt / self.tau * (U[0] - U[1] * ct - U[2] * st)
                    self.f[(v, y, x)] = loc[v] + om * (fe[v] - loc[v])

    def fields(self):
        nv = len(self.vel)
        out = [[[None] * self.nx for _ in range(self.ny)] for _ in range(4)]
        for y in range(self.ny):
            for x in range(self.nx):
                n, eps, U = self.landau(self.moments([self.f[(v, y, x)] for v in range(nv)]))
                out[0][y][x], out[1][y][x], out[2][y][x], out[3][y][x] = n, eps, U[1], U[2]
        return out
