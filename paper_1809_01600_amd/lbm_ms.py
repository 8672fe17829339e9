"""Thin ctypes binding of liblbm_ms.so (include/lbm_ms.h), same names as the C ABI.

Argument marshalling only: every step of the method runs in the library's HIP kernels.  PyTorch
provides the device workspace and the stream.  There is no fallback: if the shared library is
missing or cannot be loaded, importing the binding's functions raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_ms.so")

D2Q9, D3Q19, D2Q5, D3Q7 = 0, 1, 2, 3
BGK, TRT = 0, 1
COLLISIONS = {"bgk": BGK, "trt": TRT}
LATTICES = {"D2Q9": D2Q9, "D3Q19": D3Q19, "D2Q5": D2Q5, "D3Q7": D3Q7}
Q_OF = {"D2Q9": 9, "D3Q19": 19, "D2Q5": 5, "D3Q7": 7}
FP64, FP32, FP16, BF16 = 0, 1, 2, 3
SHIFT_GLOBAL, SHIFT_NODE = 0, 1
LOCAL_FLUX, STOICH = 0, 1
INLET_DIRICHLET, INLET_WALL = 0, 1

OK = 0
E_ARG, E_STATE, E_GEOM, E_HIP, E_DIVERGED = -1, -2, -3, -4, -5
E_NOT_CONVERGED, E_NEG_FRACTION, E_NOMEM, E_TAU_CLAMP = -6, -7, -8, -9

PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16}


class lbm_ms_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("T", ctypes.c_double), ("p", ctypes.c_double),
        ("D", ctypes.c_double * 9),
        ("nu", ctypes.c_int * 3),
        ("n_electrons", ctypes.c_int),
        ("dx", ctypes.c_double),
        ("tau_ref", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("shift_mode", ctypes.c_int),
        ("ms_mode", ctypes.c_int),
        ("inlet_mode", ctypes.c_int),
        ("eps_flux", ctypes.c_double),
        ("tau_min", ctypes.c_double),
        ("tau_max", ctypes.c_double),
        ("tile_y", ctypes.c_int),
        ("chunk_z", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("collision", ctypes.c_int),
        ("trt_lambda", ctypes.c_double),
        ("advection", ctypes.c_int),
        ("tau_flow", ctypes.c_double),
    ]


class lbm_ms_info(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double),
        ("Ct", ctypes.c_double),
        ("Dl", ctypes.c_double * 9),
        ("Q", ctypes.c_double * 2),
        ("eps_flux", ctypes.c_double),
        ("n_fluid", ctypes.c_int64),
        ("n_open_outlet", ctypes.c_int64),
        ("steps", ctypes.c_int64),
        ("q", ctypes.c_int),
        ("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int), ("chunk_z", ctypes.c_int),
        ("workspace_bytes", ctypes.c_size_t),
        ("S", ctypes.c_double * 2),
        ("n_source", ctypes.c_int64),
        ("source_x0", ctypes.c_int),
    ]


class lbm_ms_instance_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("solid", ctypes.POINTER(ctypes.c_uint8)),
        ("X_in", ctypes.c_double * 3),
        ("j_A_per_m2", ctypes.c_double),
    ]


class LbmMsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("lbm_ms status %d: %s" % (status, message))
        self.status = status


_lib = None

# (name, restype, argtypes) of every symbol in include/lbm_ms.h
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_SIGNATURES = [
    ("lbm_ms_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(lbm_ms_params)]),
    ("lbm_ms_create", ctypes.c_int, [ctypes.POINTER(lbm_ms_params), _VP, ctypes.c_size_t,
                                     ctypes.POINTER(_VP)]),
    ("lbm_ms_set_geometry", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_uint8)]),
    ("lbm_ms_get_geometry", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_uint8)]),
    ("lbm_ms_clean_geometry", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.POINTER(ctypes.c_uint8),
                                             ctypes.POINTER(ctypes.c_uint8),
                                             ctypes.POINTER(ctypes.c_int64)]),
    ("lbm_ms_work_list", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_uint8), ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                        _VP, _VP]),
    ("lbm_ms_set_bc", ctypes.c_int, [_VP, _DP, ctypes.c_double]),
    ("lbm_ms_set_source", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_double]),
    ("lbm_ms_init", ctypes.c_int, [_VP, _VP, ctypes.c_int]),
    ("lbm_ms_init_paper_profile", ctypes.c_int, [_VP]),
    ("lbm_ms_paper_profile", ctypes.c_int, [_VP, _DP]),
    ("lbm_ms_step", ctypes.c_int, [_VP, ctypes.c_int64]),
    ("lbm_ms_time_steps", ctypes.c_int, [_VP, ctypes.c_int64, _DP]),
    ("lbm_ms_residual", ctypes.c_int, [_VP, _DP]),
    ("lbm_ms_converge", ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_int64, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int64), _DP]),
    ("lbm_ms_outlet_mean", ctypes.c_int, [_VP, _DP]),
    ("lbm_ms_overpotential", ctypes.c_int, [_VP, _DP]),
    ("lbm_ms_get_fields", ctypes.c_int, [_VP, _VP, ctypes.c_int]),
    ("lbm_ms_get_populations", ctypes.c_int, [_VP, _DP]),
    ("lbm_ms_get_velocity", ctypes.c_int, [_VP, _DP]),
    ("lbm_ms_mass_balance", ctypes.c_int, [_VP, _DP, _DP, _DP]),
    ("lbm_ms_save_state", ctypes.c_int, [_VP, _VP, ctypes.POINTER(ctypes.c_size_t)]),
    ("lbm_ms_load_state", ctypes.c_int, [_VP, _VP, ctypes.c_size_t]),
    ("lbm_ms_get_info", ctypes.c_int, [_VP, ctypes.POINTER(lbm_ms_info)]),
    ("lbm_ms_lattice_info", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), _DP]),
    ("lbm_ms_tile_options", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    ("lbm_ms_set_tile", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int]),
    ("lbm_ms_batch_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(lbm_ms_params),
                                                     ctypes.POINTER(lbm_ms_instance_desc),
                                                     ctypes.c_int]),
    ("lbm_ms_batch_create", ctypes.c_int, [ctypes.POINTER(lbm_ms_params),
                                           ctypes.POINTER(lbm_ms_instance_desc), ctypes.c_int,
                                           _VP, ctypes.c_size_t, ctypes.POINTER(_VP)]),
    ("lbm_ms_batch_init", ctypes.c_int, [_VP, _VP, ctypes.c_int]),
    ("lbm_ms_batch_step", ctypes.c_int, [_VP, ctypes.c_int64]),
    ("lbm_ms_batch_time_steps", ctypes.c_int, [_VP, ctypes.c_int64, _DP]),
    ("lbm_ms_batch_converge", ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_int64, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int64), _DP,
                                             ctypes.POINTER(ctypes.c_int)]),
    ("lbm_ms_batch_overpotential", ctypes.c_int, [_VP, _DP]),
    ("lbm_ms_batch_instance", _VP, [_VP, ctypes.c_int]),
    ("lbm_ms_batch_stats", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int)]),
    ("lbm_ms_batch_set_tile", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int]),
    ("lbm_ms_batch_use_graphs", ctypes.c_int, [_VP, ctypes.c_int]),
    ("lbm_ms_batch_last_error", ctypes.c_char_p, [_VP]),
    ("lbm_ms_batch_destroy", None, [_VP]),
    ("lbm_ms_last_error", ctypes.c_char_p, [_VP]),
    ("lbm_ms_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("lbm_ms_destroy", None, [_VP]),
]

SYMBOLS = [s[0] for s in _SIGNATURES]


def lib():
    """Load liblbm_ms.so (raises when it has not been built: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblbm_ms.so is not built (run __graft_entry__.build() or "
                              "python paper_1809_01600_amd/build.py)")
        # torch first: the library links libamdhip64.so.7, and torch carries its own copy under
        # that soname; loaded first, torch's copy satisfies the library too.  Loaded the other
        # way round, the process would map two HIP runtimes, and streams or memory of one would
        # be invalid in the other.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def lattice_info(lattice: int):
    q = ctypes.c_int(0)
    lib().lbm_ms_lattice_info(lattice, ctypes.byref(q), None, None)
    e = np.zeros(3 * q.value, dtype=np.int32)
    w = np.zeros(q.value)
    lib().lbm_ms_lattice_info(lattice, ctypes.byref(q),
                              e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    return e.reshape(q.value, 3), w


def clean_geometry(lattice: str, solid: np.ndarray):
    """Host-only pore-space clean-up (no GPU needed): (cleaned uint8 mask, open outlet nodes)."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    nz, ny, nx = solid.shape
    out = np.empty_like(solid)
    n_open = ctypes.c_int64(0)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    rc = lib().lbm_ms_clean_geometry(LATTICES[lattice], nx, ny, nz,
                                     solid.ctypes.data_as(u8), out.ctypes.data_as(u8),
                                     ctypes.byref(n_open))
    if rc != OK:
        raise LbmMsError(rc, "clean_geometry")
    return out, int(n_open.value)


def work_list(lattice: str, solid: np.ndarray, tile_y: int, rows: int):
    """Host-only 2D work list of a [ny, nx] (or [1, ny, nx]) mask for launch shape (tile_y, rows):
    (tiles int32 [T, 8], entries uint32 [E]); see lbm_ms_work_list in lbm_ms.h."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1, solid.shape[-1])
    ny, nx = solid.shape
    nt, ne = ctypes.c_int64(0), ctypes.c_int64(0)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    args = (LATTICES[lattice], nx, ny, solid.ctypes.data_as(u8), int(tile_y), int(rows),
            ctypes.byref(nt), ctypes.byref(ne))
    rc = lib().lbm_ms_work_list(*args, None, None)
    if rc != OK:
        raise LbmMsError(rc, "work_list")
    tiles = np.zeros((nt.value, 8), dtype=np.int32)
    ent = np.zeros(max(ne.value, 1), dtype=np.uint32)
    rc = lib().lbm_ms_work_list(*args, tiles.ctypes.data, ent.ctypes.data)
    if rc != OK:
        raise LbmMsError(rc, "work_list")
    return tiles, ent[:ne.value]


def tile_options(lattice, precision=FP32, shift_mode: int = SHIFT_GLOBAL):
    """Compiled launch shapes (tile_y, chunk_z) for a lattice and storage mode (lattice and
    precision as constants or names)."""
    if isinstance(lattice, str):
        lattice = LATTICES[lattice]
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    ty = (ctypes.c_int * 16)()
    cz = (ctypes.c_int * 16)()
    n = lib().lbm_ms_tile_options(lattice, precision, shift_mode, ty, cz, 16)
    return [(ty[i], cz[i]) for i in range(n)]


def make_params(case, precision: int = FP64, shift_mode: int = SHIFT_GLOBAL,
                ms_mode: int = LOCAL_FLUX, inlet_mode: int = INLET_DIRICHLET,
                eps_flux: float = -1.0, tau_min: float = 0.0, tau_max: float = 0.0,
                tile_y: int = 0, chunk_z: int = 0, stream: Optional[int] = None,
                collision="bgk", trt_lambda: float = 0.0, advection: bool = False,
                tau_flow: float = 0.0) -> lbm_ms_params:
    """Marshal a physical problem description (inputs.Case) into lbm_ms_params."""
    p = lbm_ms_params()
    p.lattice = LATTICES[case.lattice]
    p.nx, p.ny, p.nz = case.nx, case.ny, case.nz
    p.T, p.p = case.T, case.p
    D = case.D_matrix().reshape(-1)
    for i in range(9):
        p.D[i] = float(D[i])
    for s in range(3):
        p.nu[s] = int(case.nu[s])
    p.n_electrons = case.n_electrons
    p.dx = case.dx
    p.tau_ref = case.tau_ref
    p.precision = precision
    p.shift_mode = shift_mode
    p.ms_mode = ms_mode
    p.inlet_mode = inlet_mode
    p.eps_flux = eps_flux
    p.tau_min, p.tau_max = tau_min, tau_max
    p.tile_y, p.chunk_z = tile_y, chunk_z
    p.stream = stream
    p.collision = COLLISIONS[collision] if isinstance(collision, str) else int(collision)
    p.trt_lambda = trt_lambda
    p.advection = 1 if advection else 0
    p.tau_flow = tau_flow
    return p


class Solver:
    """One problem on one GPU: a handle plus its torch-owned device workspace."""

    def __init__(self, case, precision="fp64", shift_mode=SHIFT_GLOBAL, ms_mode=LOCAL_FLUX,
                 inlet_mode=INLET_DIRICHLET, eps_flux=-1.0, tau_min=0.0, tau_max=0.0,
                 tile_y=0, chunk_z=0, device="cuda", set_geometry=True, set_bc=True,
                 collision="bgk", trt_lambda=0.0, advection=False, tau_flow=0.0):
        import torch
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.case = case
        self.torch_device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.torch_device)
        self.params = make_params(case, precision, shift_mode, ms_mode, inlet_mode, eps_flux,
                                  tau_min, tau_max, tile_y, chunk_z, self.stream.cuda_stream,
                                  collision, trt_lambda, advection, tau_flow)
        nbytes = lib().lbm_ms_workspace_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise LbmMsError(E_ARG, lib().lbm_ms_last_error(None).decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.torch_device)
        h = _VP()
        self._check(lib().lbm_ms_create(ctypes.byref(self.params),
                                        ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                        ctypes.byref(h)), handle=False)
        self.h = h
        self.N = case.nx * case.ny * case.nz
        self.q = Q_OF[case.lattice]
        if set_geometry:
            self.set_geometry(case.mask())
            if set_bc:
                self.set_bc(case.X_in, case.j_A_m2)

    # -- plumbing ------------------------------------------------------------------------------
    def _check(self, rc: int, handle: bool = True):
        if rc != OK:
            msg = lib().lbm_ms_status_string(rc).decode()
            if handle and getattr(self, "h", None):
                msg += ": " + lib().lbm_ms_last_error(self.h).decode()
            elif not handle:  # a failed create: the library keeps its reason per thread
                msg += ": " + lib().lbm_ms_last_error(None).decode()
            raise LbmMsError(rc, msg)
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_ms_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI, same names -------------------------------------------------------------------
    def set_geometry(self, solid: np.ndarray):
        solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        if solid.size != self.N:
            raise ValueError("mask has %d entries, expected %d" % (solid.size, self.N))
        self._check(lib().lbm_ms_set_geometry(
            self.h, solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))

    def get_geometry(self) -> np.ndarray:
        out = np.empty(self.N, dtype=np.uint8)
        self._check(lib().lbm_ms_get_geometry(self.h,
                                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out.reshape(self.case.shape)

    def set_bc(self, X_in: Sequence[float], j_A_m2: float):
        x = np.ascontiguousarray(X_in, dtype=np.float64)
        self._check(lib().lbm_ms_set_bc(self.h, _dp(x), float(j_A_m2)))

    def set_source(self, x_first: int, j_A_m2: float):
        """Reaction layer x >= x_first carrying the electrode flux of current density j (see
        lbm_ms_set_source); x_first = nx removes it."""
        self._check(lib().lbm_ms_set_source(self.h, int(x_first), float(j_A_m2)))

    def init(self, X0=None):
        """X0: None (uniform inlet composition), numpy [3, ...] (host) or torch tensor (device)."""
        if X0 is None:
            self._check(lib().lbm_ms_init(self.h, None, 0))
        elif hasattr(X0, "data_ptr"):
            assert X0.dtype.is_floating_point and X0.numel() == 3 * self.N and X0.is_contiguous()
            self._check(lib().lbm_ms_init(self.h, ctypes.c_void_p(X0.data_ptr()), 1))
        else:
            a = np.ascontiguousarray(X0, dtype=np.float64).reshape(-1)
            assert a.size == 3 * self.N
            self._check(lib().lbm_ms_init(self.h, a.ctypes.data_as(_VP), 0))

    def init_paper_profile(self):
        self._check(lib().lbm_ms_init_paper_profile(self.h))

    def paper_profile(self) -> np.ndarray:
        prof = np.zeros(2 * self.case.nx)
        self._check(lib().lbm_ms_paper_profile(self.h, _dp(prof)))
        return prof.reshape(2, self.case.nx)

    def step(self, n: int = 1):
        self._check(lib().lbm_ms_step(self.h, int(n)))

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_double(0.0)
        self._check(lib().lbm_ms_time_steps(self.h, int(n), ctypes.byref(ms)))
        return ms.value

    def residual(self) -> float:
        r = ctypes.c_double(0.0)
        self._check(lib().lbm_ms_residual(self.h, ctypes.byref(r)))
        return r.value

    def converge(self, tol: float, max_steps: int, check_every: int = 100,
                 raise_on_fail: bool = True):
        """Returns (steps, residual), or (steps, residual, status) with raise_on_fail=False."""
        steps = ctypes.c_int64(0)
        r = ctypes.c_double(0.0)
        rc = lib().lbm_ms_converge(self.h, tol, int(max_steps), int(check_every),
                                   ctypes.byref(steps), ctypes.byref(r))
        if not raise_on_fail:
            return steps.value, r.value, rc
        self._check(rc)
        return steps.value, r.value

    def outlet_mean(self) -> np.ndarray:
        x = np.zeros(3)
        self._check(lib().lbm_ms_outlet_mean(self.h, _dp(x)))
        return x

    def overpotential(self) -> float:
        e = ctypes.c_double(0.0)
        self._check(lib().lbm_ms_overpotential(self.h, ctypes.byref(e)))
        return e.value

    def get_fields(self, out=None) -> np.ndarray:
        """[3, nz, ny, nx] float64 on the host, or into a contiguous float64 torch tensor."""
        if out is not None:
            self._check(lib().lbm_ms_get_fields(self.h, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        X = np.empty(3 * self.N)
        self._check(lib().lbm_ms_get_fields(self.h, X.ctypes.data_as(_VP), 0))
        return X.reshape((3,) + self.case.shape)

    def get_velocity(self) -> np.ndarray:
        """Advective coupling: u_M [3, nz, ny, nx] in m/s (the velocity the species see)."""
        u = np.empty(3 * self.N)
        self._check(lib().lbm_ms_get_velocity(self.h, _dp(u)))
        return u.reshape((3,) + self.case.shape)

    def get_populations(self) -> np.ndarray:
        f = np.empty(2 * self.q * self.N)
        self._check(lib().lbm_ms_get_populations(self.h, _dp(f)))
        return f.reshape((2, self.q) + self.case.shape)

    def mass_balance(self):
        inv, inf, outf = np.zeros(2), np.zeros(2), np.zeros(2)
        self._check(lib().lbm_ms_mass_balance(self.h, _dp(inv), _dp(inf), _dp(outf)))
        return inv, inf, outf

    def save_state(self) -> bytes:
        n = ctypes.c_size_t(0)
        self._check(lib().lbm_ms_save_state(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(lib().lbm_ms_save_state(self.h, ctypes.cast(buf, _VP), ctypes.byref(n)))
        return buf.raw[: n.value]

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(lib().lbm_ms_load_state(self.h, ctypes.cast(buf, _VP), len(blob)))

    def get_info(self) -> lbm_ms_info:
        info = lbm_ms_info()
        self._check(lib().lbm_ms_get_info(self.h, ctypes.byref(info)))
        return info

    def set_tile(self, tile_y: int, chunk_z: int = 0):
        self._check(lib().lbm_ms_set_tile(self.h, tile_y, chunk_z))


class _InstanceView(Solver):
    """A batch member: the single-instance calls on a handle the batch owns."""

    def __init__(self, batch, k, case):  # noqa: D401  (no workspace of its own)
        self.case = case
        self.h = lib().lbm_ms_batch_instance(batch.b, k)
        self._batch = batch
        self.N = case.nx * case.ny * case.nz
        self.q = 9

    def close(self):
        self.h = None  # owned by the batch


class Batch:
    """Many 2D (D2Q9 or D2Q5) problems advanced by one launch per step (see lbm_ms_batch_* in
    lbm_ms.h)."""

    def __init__(self, cases, precision="fp32", shift_mode=SHIFT_GLOBAL, ms_mode=LOCAL_FLUX,
                 tile_y=0, eps_flux=-1.0, device="cuda", collision="bgk", trt_lambda=0.0, rows=0,
                 advection=False):
        import torch
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.cases = list(cases)
        c0 = self.cases[0]
        shared = ("lattice", "T", "p", "D12", "D13", "D23", "dx", "tau_ref", "nu", "n_electrons")
        for c in self.cases[1:]:
            for f in shared:
                if getattr(c, f) != getattr(c0, f):
                    raise ValueError("batch members must share %s" % f)
        if c0.lattice not in ("D2Q9", "D2Q5") or any(c.nz != 1 for c in self.cases):
            raise ValueError("batched solves are two-dimensional (D2Q9 or D2Q5)")
        self.stream = torch.cuda.current_stream(torch.device(device))
        self.params = make_params(c0, precision, shift_mode, ms_mode, INLET_DIRICHLET, eps_flux,
                                  0.0, 0.0, tile_y, rows, self.stream.cuda_stream, collision, trt_lambda,
                                  advection)
        n = len(self.cases)
        self._masks = [np.ascontiguousarray(c.mask(), dtype=np.uint8).reshape(-1) for c in self.cases]
        self.desc = (lbm_ms_instance_desc * n)()
        for k, c in enumerate(self.cases):
            d = self.desc[k]
            d.nx, d.ny = c.nx, c.ny
            d.solid = self._masks[k].ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
            for s_ in range(3):
                d.X_in[s_] = c.X_in[s_]
            d.j_A_per_m2 = c.j_A_m2
        nbytes = lib().lbm_ms_batch_workspace_bytes(ctypes.byref(self.params), self.desc, n)
        if nbytes == 0:
            raise LbmMsError(E_ARG, lib().lbm_ms_batch_last_error(None).decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=torch.device(device))
        b = _VP()
        rc = lib().lbm_ms_batch_create(ctypes.byref(self.params), self.desc, n,
                                       ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                       ctypes.byref(b))
        if rc != OK:
            raise LbmMsError(rc, lib().lbm_ms_status_string(rc).decode() + ": " +
                             lib().lbm_ms_batch_last_error(None).decode())
        self.b = b
        self.count = n

    def _check(self, rc):
        if rc != OK:
            raise LbmMsError(rc, lib().lbm_ms_status_string(rc).decode() + ": " +
                             lib().lbm_ms_batch_last_error(self.b).decode())

    def close(self):
        if getattr(self, "b", None):
            lib().lbm_ms_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, X0=None):
        if X0 is None:
            self._check(lib().lbm_ms_batch_init(self.b, None, 0))
        elif hasattr(X0, "data_ptr"):
            self._check(lib().lbm_ms_batch_init(self.b, ctypes.c_void_p(X0.data_ptr()), 1))
        else:
            a = np.ascontiguousarray(X0, dtype=np.float64).reshape(-1)
            self._check(lib().lbm_ms_batch_init(self.b, a.ctypes.data_as(_VP), 0))

    def step(self, n=1):
        self._check(lib().lbm_ms_batch_step(self.b, int(n)))

    def time_steps(self, n):
        """Milliseconds of n eager steps (HIP events on the batch's launch stream)."""
        ms = ctypes.c_double(0.0)
        self._check(lib().lbm_ms_batch_time_steps(self.b, int(n), ctypes.byref(ms)))
        return ms.value

    def converge(self, tol, max_steps, check_every=100, raise_on_fail=True):
        """Returns (steps per instance, residual per instance, overall status); per-instance
        statuses are kept in self.status."""
        steps = (ctypes.c_int64 * self.count)()
        r = (ctypes.c_double * self.count)()
        st = (ctypes.c_int * self.count)()
        rc = lib().lbm_ms_batch_converge(self.b, tol, int(max_steps), int(check_every), steps, r, st)
        self.status = np.array(st[:], dtype=np.int32)
        if raise_on_fail:
            self._check(rc)
        return np.array(steps[:], dtype=np.int64), np.array(r[:]), rc

    def overpotential(self):
        """Eq. 43 per instance (NaN for an instance whose state has a non-positive fraction)."""
        eta = np.full(self.count, np.nan)
        for k in range(self.count):
            try:
                eta[k] = self.instance(k).overpotential()
            except LbmMsError:
                pass
        return eta

    def instance(self, k) -> Solver:
        return _InstanceView(self, k, self.cases[k])

    def stats(self):
        a = ctypes.c_int(0)
        nf = ctypes.c_int64(0)
        t = ctypes.c_int(0)
        self._check(lib().lbm_ms_batch_stats(self.b, ctypes.byref(a), ctypes.byref(nf), ctypes.byref(t)))
        return a.value, nf.value, t.value

    def set_tile(self, tile_y, rows=0):
        self._check(lib().lbm_ms_batch_set_tile(self.b, int(tile_y), int(rows)))

    def use_graphs(self, enable=True):
        self._check(lib().lbm_ms_batch_use_graphs(self.b, 1 if enable else 0))
