"""Plain FP64 CPU oracle of the LBM / Maxwell-Stefan hot path (arXiv 1809.01600).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It shares no code with the HIP library: the
per-step arithmetic lives in ``lbm_ms_oracle.c`` (plain loops, no blocking or fusion) and the
host-side conversions below are written out again here from the paper.

Parity status of each function (what pins it is in the tests that name it):

* ``lattice_params`` (physical -> lattice units): pinned by the exact Stefan-tube steady state
  (slope of the binary linear profile equals Q / D*), and the continuum closed form.
* ``Oracle.step`` / ``run`` (Eq. 24-37): pinned by closed forms (binary linear profile, exact
  variance growth, discrete Stefan-tube chain, continuum matrix
  exponential), exact mass balance, and symmetry invariants.
* ``label`` (connectivity clean-up of the pore space): pinned against scipy.ndimage.label.
* ``overpotential`` (Eq. 43): pinned by j = 0 -> 0 and the binary linear profile.
* ``residual``: plain definition (relative L2 change per step over a window).
* ``paper_profile`` (initial field from the generalized Fick law at the electrode flux): pinned
  by its derivative matching Eq. 19 and by the augmented matrix exponential.
* Velocity sets D2Q9, D3Q19, D2Q5 and D3Q7 (``velocities``): isotropy and the D1Q3 marginal, the
  exact variance law, the discrete Stefan chain, conservation and clean-up on each.
* ``set_source`` (Eq. 27 on a reaction layer): conservation with the source, second-order
  convergence to the continuum profile with a distributed sink.
* ``set_trt`` (two-relaxation-time collision): reduction to BGK when both rates agree,
  conservation, a porous steady state independent of tau_ref.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

R_GAS = 8.3145        # J / (mol K), nomenclature of the paper
FARADAY = 96485.0     # C / mol, Eq. 39

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_ms_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_ms_oracle.so")

LOCAL_FLUX = 0
STOICH = 1


LATTICE_CODES = {"D2Q9": 0, "D3Q19": 1, "D2Q5": 2, "D3Q7": 3}


class _Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("Dl", ctypes.c_double * 9),
        ("X_in", ctypes.c_double * 2),
        ("Q", ctypes.c_double * 2),
        ("nu", ctypes.c_double * 3),
        ("inlet_wall", ctypes.c_int),
        ("ms_mode", ctypes.c_int),
        ("eps", ctypes.c_double),
        ("tau_min", ctypes.c_double), ("tau_max", ctypes.c_double),
        ("S", ctypes.c_double * 2), ("src_x0", ctypes.c_int),
        ("trt", ctypes.c_int), ("lambda_trt", ctypes.c_double),
        ("tau_flow", ctypes.c_double),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("inflow", ctypes.c_double * 2),
        ("outflow", ctypes.c_double * 2),
        ("clamp_hits", ctypes.c_long),
    ]


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (strict IEEE: no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.orc_step.argtypes = [ctypes.POINTER(_Params), u8p, dp, dp, ctypes.POINTER(_Stats)]
        L.orc_run.argtypes = [ctypes.POINTER(_Params), u8p, dp, dp, ctypes.c_long,
                              ctypes.POINTER(_Stats)]
        L.orc_collide.argtypes = [ctypes.POINTER(_Params), u8p, dp, dp, dp, dp,
                                  ctypes.POINTER(_Stats)]
        L.orc_moments.argtypes = [ctypes.POINTER(_Params), u8p, dp, dp]
        L.orc_equilibrium.argtypes = [ctypes.POINTER(_Params), u8p, dp, dp]
        L.orc_label.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, u8p]
        L.orc_label.restype = ctypes.c_long
        L.orc_step_adv.argtypes = [ctypes.POINTER(_Params), u8p, dp, dp, dp, dp, dp, dp,
                                   ctypes.POINTER(_Stats)]
        L.orc_run_adv.argtypes = [ctypes.POINTER(_Params), u8p, dp, dp, dp, dp, dp, ctypes.c_long,
                                  ctypes.POINTER(_Stats)]
        L.orc_collide_adv.argtypes = [ctypes.POINTER(_Params), u8p, dp, dp, dp, dp, dp, dp, dp,
                                      ctypes.POINTER(_Stats)]
        L.orc_flow_rest.argtypes = [ctypes.POINTER(_Params), u8p, dp]
        L.orc_num_velocities.argtypes = [ctypes.c_int]
        L.orc_velocities.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def velocities(lattice: str):
    """(e [Q,3] int, w [Q]) of the oracle's velocity set."""
    code = LATTICE_CODES[lattice]
    q = lib().orc_num_velocities(code)
    e = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    lib().orc_velocities(code, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    return e, w


def label(lattice: str, solid: np.ndarray):
    """Connectivity clean-up (fluid not linked to the inlet column becomes solid).

    Returns (cleaned uint8 mask, number of open outlet nodes)."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    nz, ny, nx = solid.shape
    out = np.empty_like(solid)
    n_out = lib().orc_label(LATTICE_CODES[lattice], nx, ny, nz, _u8(solid), _u8(out))
    return out, int(n_out)


def lattice_params(case, n_open: Optional[int] = None) -> dict:
    """Physical inputs -> lattice units.

    dt = (tau_ref - 1/2) dx^2 / (3 max D_ij) so that the fastest pair relaxes with tau_ref;
    D*_ij = D_ij dt / dx^2; electrode flux N_s = -nu_s I / (n F) (Eq. 39) with I in A/m^2;
    C_t = p / (R T) (Sec. 4.1); lattice outflow per outlet node Q_s = N_s dt / (C_t dx), scaled
    by (outlet face nodes / open outlet nodes) so the face carries the superficial current.
    """
    D = case.D_matrix()
    Dmax = max(case.D12, case.D13, case.D23)
    dt = (case.tau_ref - 0.5) * case.dx ** 2 / (3.0 * Dmax)
    Dl = D * dt / case.dx ** 2
    Ct = case.p / (R_GAS * case.T)
    I = case.j_A_cm2 * 1.0e4
    N = np.array([-case.nu[s] * I / (case.n_electrons * FARADAY) for s in range(3)])
    n_face = case.ny * case.nz
    if n_open is None:
        n_open = n_face
    scale = n_face / n_open if n_open > 0 else 0.0
    Q = N[:2] * dt / (Ct * case.dx) * scale
    return {"dt": dt, "Dl": Dl, "Ct": Ct, "N": N, "Q": Q, "n_face": n_face, "n_open": n_open}


def default_eps(Q) -> float:
    """Regularizer of the flux-norm ratio in Eq. 24: one percent of the imposed lattice flux plus
    an absolute floor, so the ratio of two vanishing flux norms tends to the stoichiometric ratio
    instead of amplifying roundoff."""
    return 1.0e-2 * float(np.max(np.abs(np.asarray(Q, dtype=float)))) + 1.0e-14


class Oracle:
    """One problem on the CPU.  State ``f`` is the pre-collision population array
    [2, Q, nz, ny, nx] (float64)."""

    def __init__(self, case, ms_mode: int = LOCAL_FLUX, inlet_wall: bool = False,
                 eps: Optional[float] = None, tau_min: float = 0.5 + 1.0e-9,
                 tau_max: float = 1.0e6,
                 clean_geometry: bool = True, Q_override=None, advection: bool = False,
                 tau_flow: float = 1.0):
        self.case = case
        self.lattice = case.lattice
        mask = case.mask()
        if clean_geometry and not inlet_wall:
            mask, n_open = label(case.lattice, mask)
            if n_open <= 0:
                raise ValueError("outlet not reachable from the inlet")
        else:
            n_open = int((mask[:, :, -1] == 0).sum())
        self.solid = np.ascontiguousarray(mask, dtype=np.uint8)
        self.n_open = n_open
        self.n_source = 0
        self.lp = lattice_params(case, n_open)
        self.e, self.w = velocities(case.lattice)
        self.q = len(self.w)
        p = _Params()
        p.lattice = LATTICE_CODES[case.lattice]
        p.nx, p.ny, p.nz = case.nx, case.ny, case.nz
        for i in range(3):
            for j in range(3):
                p.Dl[3 * i + j] = self.lp["Dl"][i, j]
        p.X_in[0], p.X_in[1] = case.X_in[0], case.X_in[1]
        Q = self.lp["Q"] if Q_override is None else np.asarray(Q_override, dtype=float)
        p.Q[0], p.Q[1] = float(Q[0]), float(Q[1])
        for s in range(3):
            p.nu[s] = float(case.nu[s])
        p.inlet_wall = 1 if inlet_wall else 0
        p.ms_mode = ms_mode
        p.eps = default_eps(Q) if eps is None else eps
        p.tau_min, p.tau_max = tau_min, tau_max
        p.S[0], p.S[1], p.src_x0 = 0.0, 0.0, case.nx  # no volumetric source
        p.trt, p.lambda_trt = 0, 0.25  # BGK unless set_trt
        p.tau_flow = tau_flow
        self.p = p
        self.N = case.nx * case.ny * case.nz
        self.f = np.zeros((2, self.q) + case.shape)
        # advective coupling (Eq. 26): the velocity model's populations, at rest until init
        self.advection = advection
        self.g = np.zeros((self.q,) + case.shape) if advection else None
        self.uprev = np.zeros((3,) + case.shape) if advection else None  # u of the last step
        self.t = 0
        self.last = _Stats()

    def set_trt(self, lam: Optional[float] = 0.25):
        """Two-relaxation-time collision with (tau_even - 1/2)(tau - 1/2) = lam; None restores
        the paper's BGK collision (Eq. 28)."""
        self.p.trt = 0 if lam is None else 1
        self.p.lambda_trt = 0.25 if lam is None else float(lam)

    def set_source(self, x_first: int, j_A_cm2: float):
        """Reaction spread uniformly over the fluid nodes of the columns x >= x_first (a functional
        layer next to the electrolyte): the source term of Eq. 27, F_a = w_a S_s, on every such
        node.  The layer's total per step equals the electrode flux of Eq. 39 at current density
        j over the whole face (the superficial current): with N_s = -nu_s I / (n F),
        S_s = -N_s dt n_face / (C_t dx n_layer).  x_first = nx removes the source."""
        if not 0 <= x_first <= self.case.nx:
            raise ValueError("x_first outside [0, nx]")
        if x_first == self.case.nx:
            self.p.S[0] = self.p.S[1] = 0.0
            self.p.src_x0 = x_first
            self.n_source = 0
            return
        n_layer = int((self.solid[:, :, x_first:] == 0).sum())
        if n_layer == 0:
            raise ValueError("no fluid node in the source layer")
        lp = lattice_params(dataclasses.replace(self.case, j_A_cm2=j_A_cm2), self.n_open)
        S = -lp["N"][:2] * lp["dt"] * lp["n_face"] / (lp["Ct"] * self.case.dx * n_layer)
        self.p.S[0], self.p.S[1] = float(S[0]), float(S[1])
        self.p.src_x0 = x_first
        self.n_source = n_layer

    # -- initial states ---------------------------------------------------------------------
    def init_uniform(self):
        X0 = np.zeros((3,) + self.case.shape)
        for s in range(3):
            X0[s] = self.case.X_in[s]
        self.init_field(X0)

    def init_field(self, X0: np.ndarray):
        """Equilibrium populations of X0 at rest (the velocity model, if any, at rho = 1, u = 0)."""
        X0 = np.ascontiguousarray(X0, dtype=np.float64)
        lib().orc_equilibrium(ctypes.byref(self.p), _u8(self.solid), _dp(X0), _dp(self.f))
        if self.advection:
            lib().orc_flow_rest(ctypes.byref(self.p), _u8(self.solid), _dp(self.g))
            self.uprev[...] = 0.0
        self.t = 0

    # -- stepping -----------------------------------------------------------------------------
    def step(self, n: int = 1):
        work = np.empty_like(self.f)
        st = _Stats()
        if self.advection:
            gwork = np.empty_like(self.g)
            rc = lib().orc_run_adv(ctypes.byref(self.p), _u8(self.solid), _dp(self.f),
                                   _dp(self.g), _dp(self.uprev), _dp(work), _dp(gwork), n,
                                   ctypes.byref(st))
        else:
            rc = lib().orc_run(ctypes.byref(self.p), _u8(self.solid), _dp(self.f), _dp(work), n,
                               ctypes.byref(st))
        if rc != 0:
            raise MemoryError("oracle step failed (%d)" % rc)
        self.t += n
        self.last = st
        return st

    def step_stats(self):
        """One step; returns (inflow[2], outflow[2], clamp_hits) of that step."""
        st = self.step(1)
        return np.array(st.inflow[:2]), np.array(st.outflow[:2]), int(st.clamp_hits)

    # -- observables ---------------------------------------------------------------------------
    def moments(self, f: Optional[np.ndarray] = None) -> np.ndarray:
        f = self.f if f is None else np.ascontiguousarray(f)
        X = np.empty((3,) + self.case.shape)
        lib().orc_moments(ctypes.byref(self.p), _u8(self.solid), _dp(f), _dp(X))
        return X

    def collide_adv(self):
        """Advective coupling: (post-collision species populations, post-collision velocity
        populations, tau [2,...], u_M [3,...] in lattice units (the two-step mean the species
        see), clamp hits) of the state."""
        fstar = np.empty_like(self.f)
        gstar = np.empty_like(self.g)
        tau = np.empty((2,) + self.case.shape)
        u = np.empty((3,) + self.case.shape)
        st = _Stats()
        lib().orc_collide_adv(ctypes.byref(self.p), _u8(self.solid), _dp(self.f), _dp(self.g),
                              _dp(self.uprev), _dp(fstar), _dp(gstar), _dp(tau), _dp(u),
                              ctypes.byref(st))
        return fstar, gstar, tau, u, int(st.clamp_hits)

    def velocity(self) -> np.ndarray:
        """Molar-averaged velocity u_M [3, nz, ny, nx] of the velocity model (lattice units)."""
        return self.collide_adv()[3]

    def collide(self):
        """(post-collision populations, tau [2,...], J [2,3,...], clamp hits) of the state."""
        fstar = np.empty_like(self.f)
        tau = np.empty((2,) + self.case.shape)
        J = np.empty((2, 3) + self.case.shape)
        st = _Stats()
        lib().orc_collide(ctypes.byref(self.p), _u8(self.solid), _dp(self.f), _dp(fstar),
                          _dp(tau), _dp(J), ctypes.byref(st))
        return fstar, tau, J, int(st.clamp_hits)

    def fluid(self) -> np.ndarray:
        return self.solid == 0

    def inventory(self) -> np.ndarray:
        X = self.moments()
        fl = self.fluid()
        return np.array([X[0][fl].sum(), X[1][fl].sum()])

    def outlet_mean(self) -> np.ndarray:
        """Mean mole fractions over the open nodes of the outlet column (species 1, 2)."""
        X = self.moments()
        col = self.fluid()[:, :, -1]
        return np.array([X[0][:, :, -1][col].mean(), X[1][:, :, -1][col].mean()])

    def overpotential(self) -> float:
        return overpotential(self.case, self.outlet_mean())


def overpotential(case, X_out) -> float:
    """Eq. 43: eta = (R T / n F) ln(X1_in X2_out / (X1_out X2_in))."""
    return (R_GAS * case.T / (case.n_electrons * FARADAY)) * np.log(
        case.X_in[0] * X_out[1] / (X_out[0] * case.X_in[1]))


def residual(X_now: np.ndarray, X_prev: np.ndarray, fluid: np.ndarray, K: int) -> float:
    """Relative L2 change per step over a window of K steps, evolved species, fluid nodes."""
    a = X_now[:2][:, fluid]
    b = X_prev[:2][:, fluid]
    return float(np.sqrt(((a - b) ** 2).sum()) / (K * np.sqrt((a ** 2).sum())))


def paper_profile(case, n_points: int) -> np.ndarray:
    """The paper's initial field (Sec. 4.1, initial settings): the flux along x equals the
    electrode flux everywhere, and the generalized Fick law (Eq. 31 with Gamma = I) is
    integrated from the inlet composition.  Returns X [3, n_points] at the node positions
    x_k = k dx (k = 0 .. n_points - 1), with the superficial (unscaled) flux.

    dX/dx = -(1/C_t) [B(X)] N  is linear in X, so the solution is the augmented matrix
    exponential of the constant system dX/dx = Phi X + phi.
    """
    from scipy.linalg import expm
    D = case.D_matrix()
    Ct = case.p / (R_GAS * case.T)
    I = case.j_A_cm2 * 1.0e4
    N = np.array([-case.nu[s] * I / (case.n_electrons * FARADAY) for s in range(3)])
    # -[B(X)] N / C_t written out as an affine map of X = (X1, X2), X3 = 1 - X1 - X2
    def rhs(X12):
        X = np.array([X12[0], X12[1], 1.0 - X12[0] - X12[1]])
        B = np.zeros((2, 2))
        for i in range(2):
            for j in range(2):
                if i == j:
                    B[i, i] = X[i] / D[i, 2] + sum(X[k] / D[i, k] for k in range(3) if k != i)
                else:
                    B[i, j] = -X[i] * (1.0 / D[i, j] - 1.0 / D[i, 2])
        return -(B @ N[:2]) / Ct
    phi = rhs(np.zeros(2))
    Phi = np.column_stack([rhs(np.array([1.0, 0.0])) - phi, rhs(np.array([0.0, 1.0])) - phi])
    A = np.zeros((3, 3))
    A[:2, :2] = Phi
    A[:2, 2] = phi
    out = np.zeros((3, n_points))
    v0 = np.array([case.X_in[0], case.X_in[1], 1.0])
    for k in range(n_points):
        v = expm(A * (k * case.dx)) @ v0
        out[0, k], out[1, k] = v[0], v[1]
        out[2, k] = 1.0 - v[0] - v[1]
    return out
