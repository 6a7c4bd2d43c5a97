"""ctypes binding of liblrdm (include/lrdm.h): argument marshalling only.

Every function takes torch tensors that already live on a ROCm device, checks
dtype / shape / contiguity, and passes raw device pointers and the current HIP
stream to the C ABI.  All arithmetic happens in the library's HIP kernels; if
the library is missing or no GPU is present the calls raise, there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrdm.so")

LRDM_OK = 0
STATUS_NAMES = {0: "LRDM_OK", -1: "LRDM_EINVAL", -2: "LRDM_ENOMEM", -3: "LRDM_EDEVICE",
                -4: "LRDM_ENOTCONV", -5: "LRDM_ENONFINITE", -6: "LRDM_EUNSUPPORTED"}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}

EXPORTED = [
    "lrdm_create", "lrdm_destroy", "lrdm_set_stream", "lrdm_set_checks", "lrdm_workspace_bytes",
    "lrdm_profile", "lrdm_profile_read",
    "lrdm_last_error", "lrdm_hamiltonian_apply", "lrdm_fermi_occupations",
    "lrdm_projected_perturbation", "lrdm_hartree_kernel", "chfsi_filter",
    "subspace_rayleigh_ritz", "density_response", "lrdm_residual_derivative",
    "density_response_backward", "density_response_batched",
    "lrdm_density", "lrdm_effective_potential", "lrdm_lowrank_step", "lrdm_set_fermi_expansion",
    "lrdm_lda_xc", "lrdm_residual_derivative_xc", "lrdm_autotune",
    "lrdm_set_eigensolver_sweeps", "lrdm_set_response_block_skip", "density_response_bz",
    "lrdm_bloch_hamiltonian_apply", "chfsi_filter_bloch", "subspace_rayleigh_ritz_bloch",
    "density_response_noalloc", "lrdm_set_backproj_layout",
]


class LrdmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class c_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("L", ctypes.c_double * 3)]


class c_occ(ctypes.Structure):
    _fields_ = [("nspin", ctypes.c_int32), ("kT", ctypes.c_double), ("n_electrons", ctypes.c_double)]


class c_system(ctypes.Structure):
    _fields_ = [("grid", c_grid), ("Psi", ctypes.c_void_p), ("eps", ctypes.c_void_p),
                ("N", ctypes.c_int32), ("occ", c_occ), ("dV", ctypes.c_void_p),
                ("r", ctypes.c_int32), ("drho", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("dmu", ctypes.c_void_p)]


class c_lowrank_params(ctypes.Structure):
    _fields_ = [("s_tol", ctypes.c_double), ("r_max", ctypes.c_int32),
                ("alpha_far", ctypes.c_double), ("alpha_near", ctypes.c_double),
                ("alpha_switch", ctypes.c_double), ("r_add_max", ctypes.c_int32)]


class c_lowrank_info(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("added", ctypes.c_int32), ("s_rel", ctypes.c_double),
                ("norm_R", ctypes.c_double), ("alpha", ctypes.c_double),
                ("norm_R_lin", ctypes.c_double)]


@dataclass(frozen=True)
class Grid:
    n: tuple    # (nx, ny, nz)
    L: tuple    # (Lx, Ly, Lz)

    @property
    def M(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def shape(self) -> tuple:
        return (self.n[2], self.n[1], self.n[0])

    def c(self) -> c_grid:
        g = c_grid()
        for d in range(3):
            g.n[d] = int(self.n[d])
            g.L[d] = float(self.L[d])
        return g


@dataclass(frozen=True)
class Occupation:
    nspin: int
    kT: float
    n_electrons: float

    def c(self) -> c_occ:
        return c_occ(int(self.nspin), float(self.kT), float(self.n_electrons))


_lib = None
_lib_lock = threading.Lock()


def library() -> ctypes.CDLL:
    """Load liblrdm.so (built in-tree by paper_2211_07894_amd.build)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2211_07894_amd.build` (no CPU fallback exists)")
            lib = ctypes.CDLL(LIB_PATH)
            vp, i32, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
            G, O = ctypes.POINTER(c_grid), ctypes.POINTER(c_occ)
            sig = {
                "lrdm_create": [ctypes.POINTER(vp), ctypes.c_int, vp, sz],
                "lrdm_destroy": [vp],
                "lrdm_set_stream": [vp, vp],
                "lrdm_set_checks": [vp, ctypes.c_int],
                "lrdm_set_fermi_expansion": [vp, i32],
                "lrdm_set_eigensolver_sweeps": [vp, i32],
                "lrdm_set_response_block_skip": [vp, f64],
                "lrdm_set_backproj_layout": [vp, i32],
                "lrdm_workspace_bytes": [vp],
                "lrdm_profile": [vp, ctypes.c_int],
                "lrdm_profile_read": [vp, ctypes.c_char_p, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)],
                "lrdm_last_error": [vp],
                "lrdm_hamiltonian_apply": [vp, G, vp, vp, vp, i32, ctypes.c_int],
                "lrdm_fermi_occupations": [vp, vp, i32, O, vp, vp, vp, vp],
                "lrdm_projected_perturbation": [vp, G, vp, i32, i32, vp, i32, ctypes.c_int, vp],
                "lrdm_hartree_kernel": [vp, G, vp, vp, i32],
                "chfsi_filter": [vp, G, vp, vp, vp, i32, ctypes.c_int, i32, f64, f64, f64],
                "subspace_rayleigh_ritz": [vp, G, vp, vp, i32, ctypes.c_int, vp],
                "density_response": [vp, G, vp, vp, i32, O, vp, i32, ctypes.c_int, vp, vp, vp],
                "density_response_bz": [vp, G, vp, vp, vp, i32, i32, O, vp, i32, ctypes.c_int,
                                        vp, vp, vp],
                "lrdm_bloch_hamiltonian_apply": [vp, G, vp, f64, f64, f64, vp, vp, i32,
                                                 ctypes.c_int],
                "chfsi_filter_bloch": [vp, G, vp, f64, f64, f64, vp, vp, i32, ctypes.c_int, i32,
                                       f64, f64, f64],
                "subspace_rayleigh_ritz_bloch": [vp, G, vp, f64, f64, f64, vp, i32, ctypes.c_int,
                                                 vp],
                "density_response_noalloc": [vp, G, vp, vp, i32, O, vp, i32, ctypes.c_int, vp, vp,
                                             vp],
                "lrdm_residual_derivative": [vp, G, vp, vp, i32, O, vp, i32, ctypes.c_int, vp],
                "density_response_backward": [vp, G, vp, vp, i32, O, vp, i32, ctypes.c_int, vp,
                                              vp, vp, vp],
                "density_response_batched": [vp, ctypes.POINTER(c_system), i32, ctypes.c_int],
                "lrdm_density": [vp, G, vp, vp, i32, O, ctypes.c_int, vp, vp, vp],
                "lrdm_effective_potential": [vp, G, vp, vp, i32, vp, vp, vp],
                "lrdm_lda_xc": [vp, G, vp, i32, vp, vp],
                "lrdm_autotune": [vp, G, i32, i32, i32, ctypes.c_int, vp, vp, vp, vp, vp],
                "lrdm_residual_derivative_xc": [vp, G, vp, vp, i32, O, vp, i32, ctypes.c_int, vp,
                                                vp],
                "lrdm_lowrank_step": [vp, G, vp, vp, i32, O, ctypes.c_int, vp,
                                      ctypes.POINTER(c_lowrank_params), i32, vp, vp, vp, vp, vp,
                                      ctypes.POINTER(c_lowrank_info)],
            }
            for name, args in sig.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
            lib.lrdm_workspace_bytes.restype = sz
            lib.lrdm_last_error.restype = ctypes.c_char_p
            _lib = lib
        return _lib


class Context:
    """One liblrdm context per (device, HIP stream)."""

    def __init__(self, device: int, stream: int, workspace_limit: int = 0):
        self.lib = library()
        self.ptr = ctypes.c_void_p()
        st = self.lib.lrdm_create(ctypes.byref(self.ptr), int(device), ctypes.c_void_p(stream),
                                  int(workspace_limit))
        if st != LRDM_OK:
            raise LrdmError(st, self.lib.lrdm_last_error(None).decode())
        self.device = device
        self.stream = stream

    def check(self, st: int):
        if st != LRDM_OK:
            raise LrdmError(st, self.lib.lrdm_last_error(self.ptr).decode())

    def set_fermi_expansion(self, depth: int):
        """0: exact Fermi-Dirac divided differences; T > 0: the recursive
        expansion of depth T in the response multiplier."""
        self.check(self.lib.lrdm_set_fermi_expansion(self.ptr, int(depth)))

    def set_eigensolver_sweeps(self, max_sweeps: int):
        """Sweep limit of the subspace eigensolver (default 40); beyond it
        subspace_rayleigh_ritz raises LRDM_ENOTCONV."""
        self.check(self.lib.lrdm_set_eigensolver_sweeps(self.ptr, int(max_sweeps)))

    def set_response_block_skip(self, tau: float):
        """Drop the response blocks whose largest Fermi multiplier entry is at
        most tau times the largest (0: form every block; default 1e-14)."""
        self.check(self.lib.lrdm_set_response_block_skip(self.ptr, float(tau)))

    def set_backproj_layout(self, layout: int):
        """BF16X3 back-projection layout: 1 = 256 points per workgroup (default),
        0 = 128 points."""
        self.check(self.lib.lrdm_set_backproj_layout(self.ptr, int(layout)))

    def set_checks(self, level: int):
        self.check(self.lib.lrdm_set_checks(self.ptr, int(level)))

    def profile(self, enable: bool):
        self.check(self.lib.lrdm_profile(self.ptr, 1 if enable else 0))

    def profile_read(self, kernel: str):
        """(total milliseconds, launches) recorded for `kernel` since its last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self.check(self.lib.lrdm_profile_read(self.ptr, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    @property
    def workspace_bytes(self) -> int:
        return int(self.lib.lrdm_workspace_bytes(self.ptr))

    def close(self):
        if self.ptr:
            self.lib.lrdm_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict = {}


def context(device=None) -> Context:
    """Context bound to the current device and its current torch stream."""
    if not torch.cuda.is_available():
        raise RuntimeError("liblrdm needs a ROCm GPU; torch.cuda.is_available() is False")
    dev = torch.cuda.current_device() if device is None else int(device)
    stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, stream)
    ctx = _contexts.get(key)
    if ctx is None:
        ctx = Context(dev, stream)
        _contexts[key] = ctx
    return ctx


def release_contexts():
    for c in list(_contexts.values()):
        c.close()
    _contexts.clear()


# ------------------------------------------------------------------ marshalling helpers
def _block_dtype(prec: str):
    return torch.float64 if prec == "fp64" else torch.float32


def _ptr(t: torch.Tensor, name: str, dtype=None, numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _prec(prec: str) -> int:
    if prec not in PREC:
        raise ValueError(f"prec must be one of {sorted(PREC)}")
    return PREC[prec]


# ------------------------------------------------------------------ single steps
def hamiltonian_apply(grid: Grid, V, X, prec="fp64", out=None):
    """Y = H X, H = -1/2 Lap_h + diag(V) (7-point periodic)."""
    N = X.shape[0]
    dt = _block_dtype(prec)
    Y = torch.empty_like(X) if out is None else out
    ctx = context(X.device.index)
    g = grid.c()
    ctx.check(ctx.lib.lrdm_hamiltonian_apply(ctx.ptr, ctypes.byref(g), _ptr(V, "V", torch.float64, grid.M),
                                             _ptr(X, "X", dt, N * grid.M), _ptr(Y, "Y", dt, N * grid.M),
                                             N, _prec(prec)))
    return Y


def fermi_occupations(eps, occ: Occupation, want_F=True):
    """mu, f, f', F for eps [nspin][N] (FP64 on the GPU)."""
    eps = eps.reshape(occ.nspin, -1)
    N = eps.shape[1]
    dev = eps.device
    mu = torch.empty(1, dtype=torch.float64, device=dev)
    f = torch.empty_like(eps)
    fp = torch.empty_like(eps)
    F = torch.empty((occ.nspin, N, N), dtype=torch.float64, device=dev) if want_F else None
    ctx = context(dev.index)
    o = occ.c()
    ctx.check(ctx.lib.lrdm_fermi_occupations(ctx.ptr, _ptr(eps, "eps", torch.float64), N, ctypes.byref(o),
                                             _ptr(mu, "mu"), _ptr(f, "f"), _ptr(fp, "fprime"),
                                             _ptr(F, "F") if F is not None else None))
    return mu, f, fp, F


def projected_perturbation(grid: Grid, Psi, dV, nspin=1, prec="fp64"):
    """Hp [r][nspin][N][N] = Psi^T diag(dV) Psi per direction and channel."""
    N = Psi.shape[-4] if Psi.dim() >= 4 else Psi.shape[-2]
    r = dV.numel() // (nspin * grid.M)
    Hp = torch.empty((r, nspin, N, N), dtype=torch.float64, device=Psi.device)
    ctx = context(Psi.device.index)
    g = grid.c()
    ctx.check(ctx.lib.lrdm_projected_perturbation(
        ctx.ptr, ctypes.byref(g), _ptr(Psi, "Psi", _block_dtype(prec), nspin * N * grid.M), N, nspin,
        _ptr(dV, "dV", torch.float64, r * nspin * grid.M), r, _prec(prec), _ptr(Hp, "Hp")))
    return Hp


def hartree_kernel(grid: Grid, u, out=None):
    """dV = 4 pi (-Lap_h)^{-1} u per direction (q = 0 removed); u [r][nz][ny][nx]."""
    r = u.numel() // grid.M
    dV = torch.empty_like(u) if out is None else out
    ctx = context(u.device.index)
    g = grid.c()
    ctx.check(ctx.lib.lrdm_hartree_kernel(ctx.ptr, ctypes.byref(g), _ptr(u, "u", torch.float64, r * grid.M),
                                          _ptr(dV, "dV", torch.float64, r * grid.M), r))
    return dV


# ------------------------------------------------------------------ hot path
def chfsi_filter(grid: Grid, V, X, degree: int, a: float, b: float, a0: float, prec="fp64", out=None):
    """Y = T_c(Hbar) X / T_c(ybar0) (scaled Chebyshev filter of degree c)."""
    N = X.shape[0]
    dt = _block_dtype(prec)
    Y = torch.empty_like(X) if out is None else out
    ctx = context(X.device.index)
    g = grid.c()
    ctx.check(ctx.lib.chfsi_filter(ctx.ptr, ctypes.byref(g), _ptr(V, "V", torch.float64, grid.M),
                                   _ptr(X, "X", dt, N * grid.M), _ptr(Y, "Y", dt, N * grid.M), N,
                                   _prec(prec), int(degree), float(a), float(b), float(a0)))
    return Y


def subspace_rayleigh_ritz(grid: Grid, V, Psi, prec="fp64", eps=None):
    """In place: filtered block -> Ritz vectors; returns eps (ascending, FP64)."""
    N = Psi.shape[0]
    e = torch.empty(N, dtype=torch.float64, device=Psi.device) if eps is None else eps
    ctx = context(Psi.device.index)
    g = grid.c()
    ctx.check(ctx.lib.subspace_rayleigh_ritz(ctx.ptr, ctypes.byref(g), _ptr(V, "V", torch.float64, grid.M),
                                             _ptr(Psi, "Psi", _block_dtype(prec), N * grid.M), N,
                                             _prec(prec), _ptr(e, "eps", torch.float64, N)))
    return e


def density_response(grid: Grid, Psi, eps, occ: Occupation, dV, prec="fp64", out=None,
                     mu=None, dmu=None):
    """drho [r][nspin][M] for dV [r][nspin][M]; returns (drho, mu [1], dmu [r])."""
    ns = occ.nspin
    N = eps.numel() // ns
    r = dV.numel() // (ns * grid.M)
    dev = Psi.device
    drho = torch.empty((r, ns) + grid.shape, dtype=torch.float64, device=dev) if out is None else out
    mu = torch.empty(1, dtype=torch.float64, device=dev) if mu is None else mu
    dmu = torch.empty(r, dtype=torch.float64, device=dev) if dmu is None else dmu
    ctx = context(dev.index)
    g = grid.c()
    o = occ.c()
    ctx.check(ctx.lib.density_response(
        ctx.ptr, ctypes.byref(g), _ptr(Psi, "Psi", _block_dtype(prec), ns * N * grid.M),
        _ptr(eps, "eps", torch.float64, ns * N), N, ctypes.byref(o),
        _ptr(dV, "dV", torch.float64, r * ns * grid.M), r, _prec(prec),
        _ptr(drho, "drho", torch.float64, r * ns * grid.M), _ptr(mu, "mu", torch.float64, 1),
        _ptr(dmu, "dmu", torch.float64, r)))
    return drho, mu, dmu


def bloch_hamiltonian_apply(grid: Grid, V, X, kvec, prec="fp64", out=None):
    """H_k X for blocks X [2][N][nz][ny][nx] (real parts, then imaginary parts)."""
    N = X.shape[1]
    Y = torch.empty_like(X) if out is None else out
    ctx = context(X.device.index)
    g = grid.c()
    ctx.check(ctx.lib.lrdm_bloch_hamiltonian_apply(
        ctx.ptr, ctypes.byref(g), _ptr(V, "V", torch.float64, grid.M), float(kvec[0]),
        float(kvec[1]), float(kvec[2]), _ptr(X, "X", _block_dtype(prec), 2 * N * grid.M),
        _ptr(Y, "Y", _block_dtype(prec), 2 * N * grid.M), N, _prec(prec)))
    return Y


def chfsi_filter_bloch(grid: Grid, V, X, kvec, degree, a, b, a0, prec="fp64", out=None):
    """The Chebyshev filter with H_k on X [2][N][nz][ny][nx]; returns Y like X."""
    N = X.shape[1]
    Y = torch.empty_like(X) if out is None else out
    ctx = context(X.device.index)
    g = grid.c()
    ctx.check(ctx.lib.chfsi_filter_bloch(
        ctx.ptr, ctypes.byref(g), _ptr(V, "V", torch.float64, grid.M), float(kvec[0]),
        float(kvec[1]), float(kvec[2]), _ptr(X, "X", _block_dtype(prec), 2 * N * grid.M),
        _ptr(Y, "Y", _block_dtype(prec), 2 * N * grid.M), N, _prec(prec), int(degree), float(a),
        float(b), float(a0)))
    return Y


def subspace_rayleigh_ritz_bloch(grid: Grid, V, Psi, kvec, prec="fp64", eps=None):
    """In place: filtered complex block Psi [2][N][nz][ny][nx] (real parts, then
    imaginary parts; float64 for fp64, float32 otherwise) -> Ritz vectors of H_k;
    returns eps (ascending, FP64)."""
    N = Psi.shape[1]
    e = torch.empty(N, dtype=torch.float64, device=Psi.device) if eps is None else eps
    ctx = context(Psi.device.index)
    g = grid.c()
    ctx.check(ctx.lib.subspace_rayleigh_ritz_bloch(
        ctx.ptr, ctypes.byref(g), _ptr(V, "V", torch.float64, grid.M), float(kvec[0]),
        float(kvec[1]), float(kvec[2]), _ptr(Psi, "Psi", _block_dtype(prec), 2 * N * grid.M), N,
        _prec(prec), _ptr(e, "eps", torch.float64, N)))
    return e


def density_response_bz(grid: Grid, Psi, eps, weights, occ: Occupation, dV, prec="fp64",
                        out=None, mu=None, dmu=None):
    """Zone-sampled response (density_response_bz): Psi [nspin][nk][2][N][M] (real
    then imaginary parts of each k-point's states), eps [nspin][nk][N], weights
    [nk], dV [r][nspin][M]; returns (drho [r][nspin][M], mu [1], dmu [r])."""
    ns = occ.nspin
    nk = weights.numel()
    N = eps.numel() // (ns * nk)
    r = dV.numel() // (ns * grid.M)
    dev = Psi.device
    drho = torch.empty((r, ns) + grid.shape, dtype=torch.float64, device=dev) if out is None else out
    mu = torch.empty(1, dtype=torch.float64, device=dev) if mu is None else mu
    dmu = torch.empty(r, dtype=torch.float64, device=dev) if dmu is None else dmu
    ctx = context(dev.index)
    g = grid.c()
    o = occ.c()
    ctx.check(ctx.lib.density_response_bz(
        ctx.ptr, ctypes.byref(g), _ptr(Psi, "Psi", _block_dtype(prec), ns * nk * 2 * N * grid.M),
        _ptr(eps, "eps", torch.float64, ns * nk * N), _ptr(weights, "weights", torch.float64, nk),
        N, nk, ctypes.byref(o), _ptr(dV, "dV", torch.float64, r * ns * grid.M), r, _prec(prec),
        _ptr(drho, "drho", torch.float64, r * ns * grid.M), _ptr(mu, "mu", torch.float64, 1),
        _ptr(dmu, "dmu", torch.float64, r)))
    return drho, mu, dmu


def residual_derivative(grid: Grid, Psi, eps, occ: Occupation, u, prec="fp64", out=None,
                        fxc=None):
    """t_k = drho[K u_k] - u_k; u, t [r][nspin][M].  K = K_c, or K_c + K_xc with
    the LDA kernel fxc [nspin][nspin][M] (lda_xc)."""
    ns = occ.nspin
    N = eps.numel() // ns
    r = u.numel() // (ns * grid.M)
    t = torch.empty_like(u) if out is None else out
    ctx = context(Psi.device.index)
    g = grid.c()
    o = occ.c()
    args = [ctx.ptr, ctypes.byref(g), _ptr(Psi, "Psi", _block_dtype(prec), ns * N * grid.M),
            _ptr(eps, "eps", torch.float64, ns * N), N, ctypes.byref(o),
            _ptr(u, "u", torch.float64, r * ns * grid.M), r, _prec(prec)]
    if fxc is None:
        ctx.check(ctx.lib.lrdm_residual_derivative(*args, _ptr(t, "t", torch.float64,
                                                                r * ns * grid.M)))
    else:
        ctx.check(ctx.lib.lrdm_residual_derivative_xc(
            *args, _ptr(fxc, "fxc", torch.float64, ns * ns * grid.M),
            _ptr(t, "t", torch.float64, r * ns * grid.M)))
    return t


def _opt_ptr(t, name, dtype, numel):
    return None if t is None else _ptr(t, name, dtype, numel)


def density_response_backward(grid: Grid, Psi, eps, occ: Occupation, dV, g_drho, prec="fp64",
                              want=("dV", "Psi", "eps")):
    """Vector-Jacobian product of density_response for dL/d(delta rho) = g_drho
    [r][nspin][M]: returns (g_dV [r][nspin][M], g_Psi like Psi, g_eps [nspin][N]);
    entries not named in `want` are None and are not computed."""
    ns = occ.nspin
    N = eps.numel() // ns
    r = dV.numel() // (ns * grid.M)
    dev = Psi.device
    g_dV = torch.empty((r, ns) + grid.shape, dtype=torch.float64, device=dev) if "dV" in want else None
    g_Psi = torch.empty_like(Psi) if "Psi" in want else None
    g_eps = torch.empty((ns, N), dtype=torch.float64, device=dev) if "eps" in want else None
    ctx = context(dev.index)
    g = grid.c()
    o = occ.c()
    ctx.check(ctx.lib.density_response_backward(
        ctx.ptr, ctypes.byref(g), _ptr(Psi, "Psi", _block_dtype(prec), ns * N * grid.M),
        _ptr(eps, "eps", torch.float64, ns * N), N, ctypes.byref(o),
        _ptr(dV, "dV", torch.float64, r * ns * grid.M), r, _prec(prec),
        _ptr(g_drho, "g_drho", torch.float64, r * ns * grid.M),
        _opt_ptr(g_dV, "g_dV", torch.float64, r * ns * grid.M),
        _opt_ptr(g_Psi, "g_Psi", _block_dtype(prec), ns * N * grid.M),
        _opt_ptr(g_eps, "g_eps", torch.float64, ns * N)))
    return g_dV, g_Psi, g_eps


def density_response_batched(systems, prec="fp32", outs=None):
    """density_response for a list of independent systems in one call (see
    density_response_batched in lrdm.h).  Each system is a dict with grid, Psi,
    eps, occ and dV (as for density_response); returns one (drho, mu, dmu) per
    system.  outs: optional list of preallocated (drho, mu, dmu)."""
    if not systems:
        raise ValueError("systems is empty")
    dev = systems[0]["Psi"].device
    arr = (c_system * len(systems))()
    res = []
    for k, sy in enumerate(systems):
        grid, occ = sy["grid"], sy["occ"]
        ns = occ.nspin
        N = sy["eps"].numel() // ns
        r = sy["dV"].numel() // (ns * grid.M)
        if outs is None:
            drho = torch.empty((r, ns) + grid.shape, dtype=torch.float64, device=dev)
            mu = torch.empty(1, dtype=torch.float64, device=dev)
            dmu = torch.empty(r, dtype=torch.float64, device=dev)
        else:
            drho, mu, dmu = outs[k]
        arr[k] = c_system(grid.c(), _ptr(sy["Psi"], "Psi", _block_dtype(prec), ns * N * grid.M),
                          _ptr(sy["eps"], "eps", torch.float64, ns * N), N, occ.c(),
                          _ptr(sy["dV"], "dV", torch.float64, r * ns * grid.M), r,
                          _ptr(drho, "drho", torch.float64, r * ns * grid.M),
                          _ptr(mu, "mu", torch.float64, 1), _ptr(dmu, "dmu", torch.float64, r))
        res.append((drho, mu, dmu))
    ctx = context(dev.index)
    ctx.check(ctx.lib.density_response_batched(ctx.ptr, arr, len(systems), _prec(prec)))
    return res


class DensityResponse(torch.autograd.Function):
    """delta rho = density_response(Psi, eps, dV) with the library's adjoint as
    backward.  Only the inputs are kept for backward (Psi, eps and dV by
    reference); H' and Gamma are recomputed there.

        drho = DensityResponse.apply(Psi, eps, dV, grid, occ, prec)
    """

    @staticmethod
    def forward(ctx, Psi, eps, dV, grid, occ, prec="fp64"):
        drho, _, _ = density_response(grid, Psi.detach(), eps.detach(), occ, dV.detach(), prec=prec)
        ctx.save_for_backward(Psi, eps, dV)
        ctx.grid, ctx.occ, ctx.prec = grid, occ, prec
        return drho

    @staticmethod
    def backward(ctx, g):
        Psi, eps, dV = ctx.saved_tensors
        want = tuple(n for n, need in zip(("Psi", "eps", "dV"), ctx.needs_input_grad[:3]) if need)
        g_dV, g_Psi, g_eps = density_response_backward(
            ctx.grid, Psi.detach(), eps.detach(), ctx.occ, dV.detach(),
            g.detach().to(torch.float64).contiguous(), prec=ctx.prec, want=want)
        if g_eps is not None:
            g_eps = g_eps.reshape(eps.shape)
        if g_dV is not None:
            g_dV = g_dV.reshape(dV.shape)
        return g_Psi, g_eps, g_dV, None, None, None



# ------------------------------------------------------------------ low-rank step and model SCF
@dataclass(frozen=True)
class LowRankParams:
    """Parameters of the low-rank step (lrdm_lowrank_params); defaults are the
    values of Sec. III A (alpha 0.1 until ||R|| goes below 2.0, then 0.5)."""
    s_tol: float = 0.3
    r_max: int = 20
    alpha_far: float = 0.1
    alpha_near: float = 0.5
    alpha_switch: float = 2.0
    r_add_max: int = 0           # 0: up to r_max; k > 0: at most k new; -1: kept ones only

    def c(self) -> c_lowrank_params:
        return c_lowrank_params(float(self.s_tol), int(self.r_max), float(self.alpha_far),
                                float(self.alpha_near), float(self.alpha_switch), int(self.r_add_max))


def density(grid: Grid, Psi, eps, occ: Occupation, prec="fp64", rho_in=None, out=None, mu=None):
    """rho [nspin][M] of Eq. (1), or the residual rho - rho_in when rho_in is
    given; returns (out, mu [1])."""
    ns = occ.nspin
    N = eps.numel() // ns
    dev = Psi.device
    out = torch.empty((ns,) + grid.shape, dtype=torch.float64, device=dev) if out is None else out
    mu = torch.empty(1, dtype=torch.float64, device=dev) if mu is None else mu
    ctx = context(dev.index)
    g = grid.c()
    o = occ.c()
    ctx.check(ctx.lib.lrdm_density(
        ctx.ptr, ctypes.byref(g), _ptr(Psi, "Psi", _block_dtype(prec), ns * N * grid.M),
        _ptr(eps, "eps", torch.float64, ns * N), N, ctypes.byref(o), _prec(prec),
        _opt_ptr(rho_in, "rho_in", torch.float64, ns * grid.M),
        _ptr(out, "out", torch.float64, ns * grid.M), _ptr(mu, "mu", torch.float64, 1)))
    return out, mu


def effective_potential(grid: Grid, V_ext, rho, out=None, vrange=None, vxc=None):
    """V_eff = V_ext + K_c sum_c rho_c [M], or with vxc [nspin][M] (lda_xc)
    V_eff [nspin][M] = that + vxc per channel; vrange (device double [2],
    optional) receives its min and max."""
    ns = rho.numel() // grid.M
    nout = ns if vxc is not None else 1
    shape = (nout,) + grid.shape if vxc is not None else grid.shape
    out = torch.empty(shape, dtype=torch.float64, device=rho.device) if out is None else out
    ctx = context(rho.device.index)
    g = grid.c()
    ctx.check(ctx.lib.lrdm_effective_potential(
        ctx.ptr, ctypes.byref(g), _ptr(V_ext, "V_ext", torch.float64, grid.M),
        _ptr(rho, "rho", torch.float64, ns * grid.M), ns,
        _opt_ptr(vxc, "vxc", torch.float64, ns * grid.M),
        _ptr(out, "V_eff", torch.float64, nout * grid.M),
        _opt_ptr(vrange, "vrange", torch.float64, 2)))
    return out


def lda_xc(grid: Grid, rho, vxc=None, fxc=None):
    """LDA potential vxc [nspin][M] and kernel fxc [nspin][nspin][M] at rho
    [nspin][M] (lrdm_lda_xc)."""
    ns = rho.numel() // grid.M
    dev = rho.device
    vxc = torch.empty((ns,) + grid.shape, dtype=torch.float64, device=dev) if vxc is None else vxc
    fxc = (torch.empty((ns, ns) + grid.shape, dtype=torch.float64, device=dev)
           if fxc is None else fxc)
    ctx = context(dev.index)
    g = grid.c()
    ctx.check(ctx.lib.lrdm_lda_xc(ctx.ptr, ctypes.byref(g),
                                  _ptr(rho, "rho", torch.float64, ns * grid.M), ns,
                                  _ptr(vxc, "vxc", torch.float64, ns * grid.M),
                                  _ptr(fxc, "fxc", torch.float64, ns * ns * grid.M)))
    return vxc, fxc


def lowrank_step(grid: Grid, Psi, eps, occ: Occupation, R, params: LowRankParams = LowRankParams(),
                 prec="fp64", rho=None, U=None, T=None, drho=None, r_keep: int = 0, fxc=None):
    """drho_bar = P^lr_r R with the adaptive rank, and rho -= alpha drho_bar when
    rho is given (lrdm_lowrank_step).  With r_keep > 0 the first r_keep rows of
    U and T are directions kept from earlier steps (LRDMA); fxc [nspin][nspin][M]
    adds the LDA kernel to K.  Returns (drho, U[:rank], T[:rank], info) with info
    a dict of rank, added, s_rel, norm_R, alpha and norm_R_lin."""
    ns = occ.nspin
    N = eps.numel() // ns
    n = ns * grid.M
    dev = Psi.device
    shape = (ns,) + grid.shape
    U = torch.empty((params.r_max,) + shape, dtype=torch.float64, device=dev) if U is None else U
    T = torch.empty((params.r_max,) + shape, dtype=torch.float64, device=dev) if T is None else T
    drho = torch.empty(shape, dtype=torch.float64, device=dev) if drho is None else drho
    info = c_lowrank_info()
    p = params.c()
    ctx = context(dev.index)
    g = grid.c()
    o = occ.c()
    ctx.check(ctx.lib.lrdm_lowrank_step(
        ctx.ptr, ctypes.byref(g), _ptr(Psi, "Psi", _block_dtype(prec), ns * N * grid.M),
        _ptr(eps, "eps", torch.float64, ns * N), N, ctypes.byref(o), _prec(prec),
        _ptr(R, "R", torch.float64, n), ctypes.byref(p), int(r_keep),
        _opt_ptr(fxc, "fxc", torch.float64, ns * ns * grid.M),
        _ptr(U, "U", torch.float64, params.r_max * n), _ptr(T, "T", torch.float64, params.r_max * n),
        _ptr(drho, "drho", torch.float64, n), _opt_ptr(rho, "rho", torch.float64, n),
        ctypes.byref(info)))
    r = int(info.rank)
    return drho, U[:r], T[:r], dict(rank=r, added=int(info.added), s_rel=float(info.s_rel),
                                    norm_R=float(info.norm_R), alpha=float(info.alpha),
                                    norm_R_lin=float(info.norm_R_lin))


def autotune(grid: Grid, N: int, nspin: int, r: int, prec="fp64", device=None):
    """Pick the projection's layout of tiles and waves and its K-split counts for
    this shape on the current context (lrdm_autotune), and in the BF16X3 form the
    back-projection layout.  Returns dict(splits=[3], variants=[3],
    ms=[shape][layout][4 candidates], backproj_layout, backproj_ms=[2]) for the
    shapes response, single direction and Gram; 0 where not tried."""
    ctx = context(device)
    g = grid.c()
    splits = (ctypes.c_int32 * 3)()
    variants = (ctypes.c_int32 * 3)()
    ms = (ctypes.c_double * 36)()
    bp = ctypes.c_int32()
    bp_ms = (ctypes.c_double * 2)()
    ctx.check(ctx.lib.lrdm_autotune(ctx.ptr, ctypes.byref(g), int(N), int(nspin), int(r),
                                    _prec(prec), ctypes.cast(splits, ctypes.c_void_p),
                                    ctypes.cast(variants, ctypes.c_void_p),
                                    ctypes.cast(ms, ctypes.c_void_p),
                                    ctypes.cast(ctypes.byref(bp), ctypes.c_void_p),
                                    ctypes.cast(bp_ms, ctypes.c_void_p)))
    return dict(splits=list(splits), variants=list(variants),
                ms=[[list(ms[12 * k + 4 * v:12 * k + 4 * v + 4]) for v in range(3)]
                    for k in range(3)],
                backproj_layout=int(bp.value), backproj_ms=list(bp_ms))
