"""A second, literal transcription of one time step of the method, node by node in plain Python
loops, used only to check the C oracle on tiny grids.

It is written from the statement of the method, not from the oracle's source, and takes its own
route wherever one exists: the velocity sets are literal tables (Eq. 2 and Eq. 9 for D2Q9, the
nineteen vectors of D3Q19 and the axis sets written out), the lattice units and the outlet flux
are derived here from the physical inputs, and the 2x2 Maxwell-Stefan systems are solved with
numpy.linalg.solve instead of Cramer's rule.

State: pre-collision populations f[s][a][n] (s = 0, 1: H2, H2O; the inert Ar is the balance),
n = (z * ny + y) * nx + x.  One step:

  1. moments X_s = sum_a f_a^s (Eq. 29 makes f a mole-fraction distribution), X_3 = 1 - X_1 - X_2
     (Sec. 3.2, closure of the (n-1) formulation);
  2. gradients per axis: central difference between two fluid neighbours, one-sided when one
     neighbour is solid or beyond the x faces (so forward at the inlet column, Eq. 35), zero when
     neither is fluid; at the outlet column the x gradient is Eq. 37's -[B] J with the imposed
     flux; y and z wrap periodically;
  3. [B] of Eq. 32 and the generalized Fick fluxes J = -[B]^-1 grad X (Eq. 33-34, Gamma = I);
     N = J since the total flux vanishes (Eq. 21 with u_M = 0);
  4. Eq. 24 with the flux vectors replaced by signed norms: N_i = -sgn(nu_i) |N_i|, the norm ratio
     regularized by eps |nu| (or fixed at |nu_j| / |nu_i| in the stoichiometric variant);
  5. tau_i = 3 D*_i + 1/2 (Eq. 25, c_s^2 = 1/3), clamped to [tau_min, tau_max];
  6. BGK collision toward w_a X_s (Eq. 28 with Eq. 29);
  7. streaming by pull: from r - e_a if that node exists and is fluid, else half-way bounce-back
     f_a(r) = f*_abar(r) (Sec. 3.3) -- except that a source beyond the x faces is a boundary link
     whatever the in-domain neighbours are;
  8. inlet links: f_a = (w_a + w_abar) X_in - f_abar, with f_abar the value after step 7 (Eq. 36
     at the boundary node); outlet links: f_a = f*_abar - (w_abar / W_n) Q_s, W_n the weight sum
     of the velocities with e_x = +1, Q_s the electrode flux of Eq. 39 per open outlet node in
     lattice units.
"""

from __future__ import annotations

import math

import numpy as np

R_GAS = 8.3145      # J/(mol K), Sec. 4.1
FARADAY = 96485.0   # C/mol, Eq. 39

# (e, w) tables, written out
VELOCITIES = {
    # Eq. 2 order: rest, the four axis links counter-clockwise from +x, then the diagonals from
    # (1, 1) counter-clockwise; Eq. 9 weights
    "D2Q9": ([(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
              (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)],
             [4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36]),
    "D2Q5": ([(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0)],
             [1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6]),
    "D3Q19": ([(0, 0, 0),
               (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
               (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
               (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
               (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)],
              [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12),
    "D3Q7": ([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
             [0.0] + [1 / 6] * 6),
}


class LiteralStep:
    """Tiny-grid stepper.  mask: uint8 [nz, ny, nx] (1 = solid), used as given."""

    def __init__(self, case, mask, ms_mode_stoich: bool, eps: float,
                 tau_min: float = 0.5 + 1e-9, tau_max: float = 1e6, advection: bool = False,
                 tau_flow: float = 1.0):
        self.nx, self.ny, self.nz = case.nx, case.ny, case.nz
        self.dims = 3 if case.lattice.startswith("D3") else 2
        e, w = VELOCITIES[case.lattice]
        self.e = [list(v) for v in e]
        self.w = list(w)
        self.q = len(self.w)
        self.opp = [self.e.index([-c for c in v]) for v in self.e]
        self.Wn = sum(wa for v, wa in zip(self.e, self.w) if v[0] == 1)
        self.solid = [int(v) for v in np.asarray(mask).reshape(-1)]
        self.N = self.nx * self.ny * self.nz
        # lattice units: the fastest pair relaxes with tau_ref
        D = [[0.0, case.D12, case.D13], [case.D12, 0.0, case.D23], [case.D13, case.D23, 0.0]]
        dt = (case.tau_ref - 0.5) * case.dx ** 2 / (3.0 * max(case.D12, case.D13, case.D23))
        self.Dl = [[D[i][j] * dt / case.dx ** 2 for j in range(3)] for i in range(3)]
        # electrode flux (Eq. 39), superficial: scaled to the open outlet nodes
        Ct = case.p / (R_GAS * case.T)
        I = case.j_A_cm2 * 1e4
        n_face = self.ny * self.nz
        n_open = sum(1 for z in range(self.nz) for y in range(self.ny)
                     if not self.solid[self._n(self.nx - 1, y, z)])
        self.Q = [-case.nu[s] * I / (case.n_electrons * FARADAY) * dt / (Ct * case.dx)
                  * n_face / n_open for s in range(2)]
        self.nu = list(case.nu)
        self.X_in = list(case.X_in)
        self.stoich = ms_mode_stoich
        self.eps = eps
        self.tau_min, self.tau_max = tau_min, tau_max
        self.advection = advection
        self.tau_flow = tau_flow

    def _n(self, x, y, z):
        return (z * self.ny + y) * self.nx + x

    def _fluid(self, x, y, z):
        """Existing fluid node? x does not wrap, y and z do."""
        if x < 0 or x >= self.nx:
            return False
        return not self.solid[self._n(x, y % self.ny, z % self.nz)]

    def equilibrium(self, X0):
        """f_a = w_a X0_s on fluid nodes; X0 [3][nz][ny][nx]."""
        X0 = np.asarray(X0)
        f = [[[0.0] * self.N for _ in range(self.q)] for _ in range(2)]
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    n = self._n(x, y, z)
                    if self.solid[n]:
                        continue
                    for s in range(2):
                        for a in range(self.q):
                            f[s][a][n] = self.w[a] * float(X0[s, z, y, x])
        return f

    def moments(self, f):
        X = [[0.0] * self.N for _ in range(3)]
        for n in range(self.N):
            if self.solid[n]:
                continue
            for s in range(2):
                total = 0.0
                for a in range(self.q):
                    total += f[s][a][n]
                X[s][n] = total
            X[2][n] = 1.0 - X[0][n] - X[1][n]
        return X

    def _B(self, Xn):
        """Eq. 32 for three species, species 3 the balance."""
        Dl = self.Dl
        B = [[0.0, 0.0], [0.0, 0.0]]
        for i in range(2):
            B[i][i] = Xn[i] / Dl[i][2] + sum(Xn[k] / Dl[i][k] for k in range(3) if k != i)
            j = 1 - i
            B[i][j] = -Xn[i] * (1.0 / Dl[i][j] - 1.0 / Dl[i][2])
        return B

    def collide(self, f):
        """Steps 1-6: post-collision populations and the relaxation times."""
        X = self.moments(f)
        fs = [[[0.0] * self.N for _ in range(self.q)] for _ in range(2)]
        taus = [[0.0] * self.N for _ in range(2)]
        hits = 0
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    n = self._n(x, y, z)
                    if self.solid[n]:
                        continue
                    Xn = [X[0][n], X[1][n], X[2][n]]
                    B = self._B(Xn)
                    grad = [[0.0] * 3 for _ in range(2)]
                    pos = [x, y, z]
                    for d in range(self.dims):
                        if d == 0 and x == self.nx - 1:
                            # Eq. 37: the imposed flux fixes the gradient, -[B] Q
                            for s in range(2):
                                grad[s][0] = -(B[s][0] * self.Q[0] + B[s][1] * self.Q[1])
                            continue
                        up = list(pos)
                        dn = list(pos)
                        up[d] += 1
                        dn[d] -= 1
                        fu = self._fluid(*up)
                        fd = self._fluid(*dn)
                        for s in range(2):
                            c = X[s][n]
                            vu = X[s][self._n(up[0], up[1] % self.ny, up[2] % self.nz)] if fu else None
                            vd = X[s][self._n(dn[0], dn[1] % self.ny, dn[2] % self.nz)] if fd else None
                            if fu and fd:
                                grad[s][d] = (vu - vd) / 2.0
                            elif fu:
                                grad[s][d] = vu - c
                            elif fd:
                                grad[s][d] = c - vd
                            else:
                                grad[s][d] = 0.0
                    J = [[0.0] * 3 for _ in range(2)]
                    Bm = np.array(B)
                    for d in range(self.dims):
                        sol = np.linalg.solve(Bm, np.array([grad[0][d], grad[1][d]]))
                        J[0][d] = -float(sol[0])
                        J[1][d] = -float(sol[1])
                    norm = [math.sqrt(sum(J[s][d] ** 2 for d in range(self.dims))) for s in range(2)]
                    sigma = [(-1.0 if v > 0 else (1.0 if v < 0 else 0.0)) for v in self.nu]
                    for i in range(2):
                        inv = 0.0
                        for j in range(3):
                            if j == i:
                                continue
                            if sigma[j] == 0.0:
                                term = Xn[j]
                            else:
                                if self.stoich:
                                    rho = abs(self.nu[j]) / abs(self.nu[i])
                                else:
                                    rho = (norm[j] + self.eps * abs(self.nu[j])) / \
                                          (norm[i] + self.eps * abs(self.nu[i]))
                                term = Xn[j] - Xn[i] * (sigma[j] / sigma[i]) * rho
                            inv += term / self.Dl[i][j]
                        tau = 3.0 / inv + 0.5
                        if not tau >= self.tau_min:
                            tau = self.tau_min
                            hits += 1
                        elif tau > self.tau_max:
                            tau = self.tau_max
                            hits += 1
                        taus[i][n] = tau
                    for s in range(2):
                        for a in range(self.q):
                            fa = f[s][a][n]
                            fs[s][a][n] = fa - (fa - self.w[a] * Xn[s]) / taus[s][n]
        return fs, taus, hits

    def step(self, f):
        """Steps 1-8: f^t -> f^{t+1}; also returns the inflow and outflow of the step."""
        fs, _, _ = self.collide(f)
        fn = [[[0.0] * self.N for _ in range(self.q)] for _ in range(2)]
        inflow = [0.0, 0.0]
        outflow = [0.0, 0.0]
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    n = self._n(x, y, z)
                    if self.solid[n]:
                        continue
                    inlet_links, outlet_links = [], []
                    for a in range(self.q):
                        sx, sy, sz = x - self.e[a][0], y - self.e[a][1], z - self.e[a][2]
                        if sx < 0:
                            inlet_links.append(a)
                        elif sx >= self.nx:
                            outlet_links.append(a)
                        elif self.solid[self._n(sx, sy % self.ny, sz % self.nz)]:
                            for s in range(2):
                                fn[s][a][n] = fs[s][self.opp[a]][n]
                        else:
                            m = self._n(sx, sy % self.ny, sz % self.nz)
                            for s in range(2):
                                fn[s][a][n] = fs[s][a][m]
                    for a in inlet_links:
                        b = self.opp[a]
                        for s in range(2):
                            fn[s][a][n] = (self.w[a] + self.w[b]) * self.X_in[s] - fn[s][b][n]
                            inflow[s] += fn[s][a][n] - fs[s][b][n]
                    for a in outlet_links:
                        b = self.opp[a]
                        for s in range(2):
                            fn[s][a][n] = fs[s][b][n] - (self.w[b] / self.Wn) * self.Q[s]
                            outflow[s] += fs[s][b][n] - fn[s][a][n]
        return fn, inflow, outflow

    def to_array(self, f):
        """[2][Q][nz][ny][nx] numpy copy, velocity order of this module."""
        return np.array(f).reshape((2, self.q, self.nz, self.ny, self.nx))

    # -- advective coupling (Eq. 26, second LB model for u_M) --------------------------------
    #
    # State (f, g, u_prev): species populations, the velocity model's populations (Stokes-limit
    # equilibrium w_a (rho + 3 e_a . u), u = sum e_a g_a, BGK with tau_flow), and the velocity of
    # the previous step.  The species relax toward w_a X (1 + 3 e_a . u_M) with u_M the mean
    # velocity of this step and the last; Eq. 24 takes the diffusive fluxes J (Eq. 20), J_3 = -J_1
    # - J_2, ratios J_j / J_i as projections regularized toward the 1D steady ratio
    # (-nu_j - X_j Nt) / (-nu_i - X_i Nt), Nt = -(nu_1 + nu_2 + nu_3); Eq. 37's outlet gradient
    # takes J_s = Q_s - X_s (Q_1 + Q_2).  The velocity model streams like a species whose inlet
    # value is 1 and whose outlet flux is Q_1 + Q_2.

    def flow_rest(self):
        g = [[0.0] * self.N for _ in range(self.q)]
        for n in range(self.N):
            if not self.solid[n]:
                for a in range(self.q):
                    g[a][n] = self.w[a]
        return g, [[0.0] * self.N for _ in range(3)]

    def step_adv(self, f, g, uprev):
        X = self.moments(f)
        Qt = self.Q[0] + self.Q[1]
        nt = -sum(self.nu)
        fs = [[[0.0] * self.N for _ in range(self.q)] for _ in range(2)]
        gs = [[0.0] * self.N for _ in range(self.q)]
        ucur = [[0.0] * self.N for _ in range(3)]
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    n = self._n(x, y, z)
                    if self.solid[n]:
                        continue
                    rho = sum(g[a][n] for a in range(self.q))
                    u = [sum(self.e[a][d] * g[a][n] for a in range(self.q)) for d in range(3)]
                    um = [(u[d] + uprev[d][n]) / 2.0 for d in range(3)]
                    for d in range(3):
                        ucur[d][n] = u[d]
                    Xn = [X[0][n], X[1][n], X[2][n]]
                    B = self._B(Xn)
                    grad = [[0.0] * 3 for _ in range(2)]
                    pos = [x, y, z]
                    for d in range(self.dims):
                        if d == 0 and x == self.nx - 1:
                            Jb = [self.Q[0] - Xn[0] * Qt, self.Q[1] - Xn[1] * Qt]
                            for s_ in range(2):
                                grad[s_][0] = -(B[s_][0] * Jb[0] + B[s_][1] * Jb[1])
                            continue
                        up, dn = list(pos), list(pos)
                        up[d] += 1
                        dn[d] -= 1
                        fu, fd = self._fluid(*up), self._fluid(*dn)
                        for s_ in range(2):
                            c = X[s_][n]
                            vu = X[s_][self._n(up[0], up[1] % self.ny, up[2] % self.nz)] if fu else None
                            vd = X[s_][self._n(dn[0], dn[1] % self.ny, dn[2] % self.nz)] if fd else None
                            if fu and fd:
                                grad[s_][d] = (vu - vd) / 2.0
                            elif fu:
                                grad[s_][d] = vu - c
                            elif fd:
                                grad[s_][d] = c - vd
                    Bm = np.array(B)
                    J = [[0.0] * 3 for _ in range(3)]
                    for d in range(self.dims):
                        sol = np.linalg.solve(Bm, np.array([grad[0][d], grad[1][d]]))
                        J[0][d], J[1][d] = -float(sol[0]), -float(sol[1])
                        J[2][d] = -J[0][d] - J[1][d]
                    taus = [0.0, 0.0]
                    for i in range(2):
                        inv = 0.0
                        for j in range(3):
                            if j == i:
                                continue
                            r = (-self.nu[j] - Xn[j] * nt) / (-self.nu[i] - Xn[i] * nt)
                            if not self.stoich:
                                dot = sum(J[j][d] * J[i][d] for d in range(self.dims))
                                nn = sum(J[i][d] * J[i][d] for d in range(self.dims))
                                r = (dot + self.eps ** 2 * r) / (nn + self.eps ** 2)
                            inv += (Xn[j] - Xn[i] * r) / self.Dl[i][j]
                        taus[i] = min(max(3.0 / inv + 0.5, self.tau_min), self.tau_max)
                    for a in range(self.q):
                        em = sum(self.e[a][d] * um[d] for d in range(3))
                        eu = sum(self.e[a][d] * u[d] for d in range(3))
                        for s_ in range(2):
                            feq = self.w[a] * Xn[s_] * (1.0 + 3.0 * em)
                            fs[s_][a][n] = f[s_][a][n] - (f[s_][a][n] - feq) / taus[s_]
                        geq = self.w[a] * (rho + 3.0 * eu)
                        gs[a][n] = g[a][n] - (g[a][n] - geq) / self.tau_flow
        fn = self._stream(fs, [self.X_in[0], self.X_in[1]], self.Q)
        gn = self._stream([gs], [1.0], [Qt])[0]
        return fn, gn, ucur

    def _stream(self, fs, inlet, Q):
        """Pull with bounce-back and the x-face rules for a list of fields."""
        k = len(fs)
        fn = [[[0.0] * self.N for _ in range(self.q)] for _ in range(k)]
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    n = self._n(x, y, z)
                    if self.solid[n]:
                        continue
                    il, ol = [], []
                    for a in range(self.q):
                        sx, sy, sz = x - self.e[a][0], y - self.e[a][1], z - self.e[a][2]
                        if sx < 0:
                            il.append(a)
                        elif sx >= self.nx:
                            ol.append(a)
                        elif self.solid[self._n(sx, sy % self.ny, sz % self.nz)]:
                            for s_ in range(k):
                                fn[s_][a][n] = fs[s_][self.opp[a]][n]
                        else:
                            m = self._n(sx, sy % self.ny, sz % self.nz)
                            for s_ in range(k):
                                fn[s_][a][n] = fs[s_][a][m]
                    for a in il:
                        b = self.opp[a]
                        for s_ in range(k):
                            fn[s_][a][n] = (self.w[a] + self.w[b]) * inlet[s_] - fn[s_][b][n]
                    for a in ol:
                        b = self.opp[a]
                        for s_ in range(k):
                            fn[s_][a][n] = fs[s_][b][n] - (self.w[b] / self.Wn) * Q[s_]
        return fn

