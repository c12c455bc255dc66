"""ctypes binding of libmpr.so (include/mpr.h).  Argument marshalling only: every function here validates tensor
placement/dtype, allocates the outputs and the workspace the C ABI asks for, and calls the entry point of the same
name on torch's current HIP stream.  There is no CPU fallback: without the built library every call raises."""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmpr.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "mpr.h")

MPR_OK = 0
MPR_WARN_NOT_CONVERGED = 8
_STATUS = {0: "MPR_OK", 1: "MPR_ERR_INVALID_ARG", 2: "MPR_ERR_SHAPE", 3: "MPR_ERR_NO_SAMPLES",
           4: "MPR_ERR_NO_SAMPLE_BONDS", 5: "MPR_ERR_NONFINITE_INPUT", 6: "MPR_ERR_WORKSPACE_TOO_SMALL",
           7: "MPR_ERR_HIP", 8: "MPR_WARN_NOT_CONVERGED"}
INIT_RANDOM, INIT_BLOCK_MEAN = 0, 1
STOP_FIXED, STOP_AUTO, STOP_AUTO_CHAIN = 0, 1, 2
T_BLOCK, T_SITE = 0, 1
ORDER_SC, ORDER_DC = 0, 1
SWEEP_AUTO, SWEEP_TILES, SWEEP_LANES = 0, 1, 2
COUPLING_ISOTROPIC, COUPLING_DIRECTIONAL = 0, 1


class MprError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class mpr_sim_config(ctypes.Structure):
    _fields_ = [("q", ctypes.c_float), ("J", ctypes.c_float), ("n_real", ctypes.c_int32),
                ("real_offset", ctypes.c_int32), ("init_mode", ctypes.c_int32), ("stop_mode", ctypes.c_int32),
                ("n_eq", ctypes.c_int32), ("n_samp", ctypes.c_int32), ("n_fit", ctypes.c_int32),
                ("n_f", ctypes.c_int32), ("n_max", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("scene_id", ctypes.c_uint32), ("t_mode", ctypes.c_int32), ("order", ctypes.c_int32),
                ("sweep_kernel", ctypes.c_int32), ("coupling", ctypes.c_int32)]


@dataclass
class SimConfig:
    """Python mirror of mpr_sim_config (defaults: the paper's n_fit = 20, n_f = 5)."""
    q: float = 0.5
    J: float = 1.0
    n_real: int = 1
    real_offset: int = 0
    init_mode: int = INIT_BLOCK_MEAN
    stop_mode: int = STOP_AUTO
    n_eq: int = 50
    n_samp: int = 1
    n_fit: int = 20
    n_f: int = 5
    n_max: int = 1000
    seed: int = 0
    scene_id: int = 0
    t_mode: int = T_BLOCK       # T_BLOCK: one temperature per block; T_SITE: one per site (SST)
    order: int = ORDER_SC       # ORDER_SC single checkerboard; ORDER_DC double checkerboard over the blocks
    sweep_kernel: int = SWEEP_AUTO  # SWEEP_TILES / SWEEP_LANES force the sweep kernel (same chains either way)
    coupling: int = COUPLING_ISOTROPIC  # COUPLING_DIRECTIONAL: T_blocks = [Tx of the blocks, Ty of the blocks]

    def to_c(self) -> mpr_sim_config:
        return mpr_sim_config(self.q, self.J, self.n_real, self.real_offset, self.init_mode, self.stop_mode,
                              self.n_eq, self.n_samp, self.n_fit, self.n_f, self.n_max, self.seed, self.scene_id,
                              self.t_mode, self.order, self.sweep_kernel, self.coupling)


def _check_T(T_blocks, H, W, lb_h, lb_w, cfg: "SimConfig"):
    need = H * W if cfg.t_mode == T_SITE else ((H + lb_h - 1) // lb_h) * ((W + lb_w - 1) // lb_w)
    if cfg.coupling == COUPLING_DIRECTIONAL:
        need *= 2
    if T_blocks.numel() != need:
        raise ValueError(f"T_blocks has {T_blocks.numel()} entries, the grid and t_mode need {need}")


class mpr_scene(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int64), ("W", ctypes.c_int64), ("lb_h", ctypes.c_int32), ("lb_w", ctypes.c_int32),
                ("scene_id", ctypes.c_uint32), ("t", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("T_blocks", ctypes.c_void_p), ("state", ctypes.c_void_p), ("acc", ctypes.c_void_p),
                ("energy", ctypes.c_void_p)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f32 = ctypes.c_float
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t

_SIGS = {
    "mpr_abi_version": ([], _i32),
    "mpr_last_error": ([], ctypes.c_char_p),
    "mpr_map_workspace_bytes": ([_i64, _i64], _sz),
    "mpr_map_angles": ([_vp, _vp, _i64, _i64, _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
    "mpr_block_stats_workspace_bytes": ([_i64, _i64, _i32, _i32], _sz),
    "mpr_block_stats": ([_vp, _vp, _i64, _i64, _i32, _i32, _f32, _f32, _vp, _vp, _vp, _vp, _vp, _sz, _vp],
                        ctypes.c_int),
    "mpr_reference_curve_workspace_bytes": ([_i32, _i32], _sz),
    "mpr_reference_curve": ([_f32, _vp, _i32, _i32, _i32, _i32, _u64, _vp, _vp, _sz, _vp], ctypes.c_int),
    "mpr_calibrate_workspace_bytes": ([_i64, _i64, _i32, _i32], _sz),
    "mpr_calibrate_temperature": ([_vp, _vp, _i64, _i64, _i32, _i32, _f32, _f32, _vp, _vp, _i32, _vp, _vp, _vp, _vp,
                                   _sz, _vp], ctypes.c_int),
    "mpr_calibrate_temperature_noalloc": ([_vp, _vp, _i64, _i64, _i32, _i32, _f32, _f32, _vp, _vp, _i32, _vp, _vp,
                                           _vp, _vp], ctypes.c_int),
    "mpr_calibrate_directional": ([_vp, _vp, _i64, _i64, _i32, _i32, _f32, _f32, _vp, _vp, _i32, _vp, _vp, _vp, _sz,
                                   _vp], ctypes.c_int),
    "mpr_simulate_workspace_bytes": ([_i64, _i64, _i32, _i32, ctypes.POINTER(mpr_sim_config)], _sz),
    "mpr_simulate": ([_vp, _vp, _i64, _i64, _vp, _i32, _i32, ctypes.POINTER(mpr_sim_config), _vp, _vp, _vp,
                      ctypes.POINTER(_i32), _vp, _sz, _vp], ctypes.c_int),
    "mpr_sweep_workspace_bytes": ([_i64, _i64, _i32, _i32, ctypes.POINTER(mpr_sim_config)], _sz),
    "mpr_sweep": ([_vp, _vp, _vp, _i64, _i64, _vp, _i32, _i32, ctypes.POINTER(mpr_sim_config), _i32, _i32, _vp, _vp,
                   _sz, _vp], ctypes.c_int),
    "mpr_predict": ([_vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp, _vp], ctypes.c_int),
    "mpr_simulate_batched_workspace_bytes": ([ctypes.POINTER(mpr_scene), _i32, ctypes.POINTER(mpr_sim_config)], _sz),
    "mpr_simulate_batched": ([ctypes.POINTER(mpr_scene), _i32, ctypes.POINTER(mpr_sim_config), _i32,
                              ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32), _vp, _sz, _vp],
                             ctypes.c_int),
    "mpr_block_energy_workspace_bytes": ([_i64, _i64, _i32, _i32, _i32], _sz),
    "mpr_block_energy": ([_vp, _vp, _i64, _i64, _i32, _i32, _f32, _f32, _i32, _vp, _vp, _sz, _vp], ctypes.c_int),
    "mpr_temperature_grad_workspace_bytes": ([_i64, _i64, _i32], _sz),
    "mpr_temperature_grad": ([_vp, _vp, _vp, _vp, _i64, _i64, _i32, _i64, _vp, _vp, _vp, _vp, _sz, _vp],
                             ctypes.c_int),
    "mpr_validate_workspace_bytes": ([_i64], _sz),
    "mpr_validate": ([_vp, _vp, _vp, _i64, _vp, _vp, _sz, _vp], ctypes.c_int),
    "mpr_probe_instruction_rates_workspace_bytes": ([], _sz),
    "mpr_sst_temperatures_workspace_bytes": ([_i64, _i64], _sz),
    "mpr_sst_temperatures": ([_vp, _i64, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _sz, _vp], ctypes.c_int),
    "mpr_probe_instruction_rates": ([_vp, _i32, _vp, _vp, _sz, _vp], ctypes.c_int),
    "mpr_calibrate3d_workspace_bytes": ([_i64, _i64, _i64, _i32, _i32, _i32], _sz),
    "mpr_calibrate_temperature3d": ([_vp, _vp, _i64, _i64, _i64, _i32, _i32, _i32, _f32, _f32, _vp, _vp, _i32, _vp,
                                     _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
    "mpr_reference_curve3d_workspace_bytes": ([_i32, _i32], _sz),
    "mpr_reference_curve3d": ([_f32, _vp, _i32, _i32, _i32, _i32, _u64, _vp, _vp, _sz, _vp], ctypes.c_int),
    "mpr_simulate3d_workspace_bytes": ([_i64, _i64, _i64, _i32, _i32, _i32, ctypes.POINTER(mpr_sim_config)], _sz),
    "mpr_simulate3d": ([_vp, _vp, _i64, _i64, _i64, _vp, _i32, _i32, _i32, ctypes.POINTER(mpr_sim_config), _vp, _vp,
                        _vp, ctypes.POINTER(_i32), _vp, _sz, _vp], ctypes.c_int),
}


def header_symbols() -> list[str]:
    """Names of the functions declared in include/mpr.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpr_[a-z0-9_]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int, allow_warn: bool = False) -> int:
    if status == MPR_OK or (allow_warn and status == MPR_WARN_NOT_CONVERGED):
        return status
    raise MprError(status, lib().mpr_last_error().decode())


def _p(t):
    return None if t is None else _vp(t.data_ptr())


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _hw(x: torch.Tensor):
    if x.dim() != 2:
        raise ValueError("grids are 2-D [H, W]")
    return int(x.shape[0]), int(x.shape[1])


# ---------------------------------------------------------------------------------------------------------------

def mpr_map_angles(z: torch.Tensor, mask: torch.Tensor):
    _dev(z, torch.float32, "z")
    _dev(mask, torch.uint8, "mask")
    H, W = _hw(z)
    t = torch.empty_like(z)
    rng = torch.empty(2, dtype=torch.float64, device=z.device)
    ws = _ws(lib().mpr_map_workspace_bytes(H, W), z.device)
    _check(lib().mpr_map_angles(_p(z), _p(mask), H, W, _p(t), _p(rng), _p(ws), ws.numel(), _stream()))
    return t, rng


def mpr_block_stats(t, mask, lb_h, lb_w, q=0.5, J=1.0):
    _dev(t, torch.float32, "t")
    _dev(mask, torch.uint8, "mask")
    H, W = _hw(t)
    nby, nbx = -(-H // lb_h), -(-W // lb_w)
    dev = t.device
    S = torch.empty(nby * nbx, dtype=torch.float64, device=dev)
    N = torch.empty(nby * nbx, dtype=torch.int32, device=dev)
    Ts = torch.empty(nby * nbx, dtype=torch.float64, device=dev)
    No = torch.empty(nby * nbx, dtype=torch.int32, device=dev)
    ws = _ws(lib().mpr_block_stats_workspace_bytes(H, W, lb_h, lb_w), dev)
    _check(lib().mpr_block_stats(_p(t), _p(mask), H, W, lb_h, lb_w, q, J, _p(S), _p(N), _p(Ts), _p(No), _p(ws),
                                 ws.numel(), _stream()))
    return S, N, Ts, No


def mpr_reference_curve(T_grid: torch.Tensor, L: int = 128, n_therm: int = 1000, n_meas: int = 2000,
                        seed: int = 0, q: float = 0.5):
    _dev(T_grid, torch.float32, "T_grid")
    nT = int(T_grid.numel())
    e = torch.empty(nT, dtype=torch.float64, device=T_grid.device)
    ws = _ws(lib().mpr_reference_curve_workspace_bytes(nT, L), T_grid.device)
    _check(lib().mpr_reference_curve(q, _p(T_grid), nT, L, n_therm, n_meas, seed, _p(e), _p(ws), ws.numel(),
                                     _stream()))
    return e


def mpr_calibrate_temperature(t, mask, lb_h, lb_w, curve_T, curve_e, q=0.5, J=1.0):
    _dev(t, torch.float32, "t")
    _dev(mask, torch.uint8, "mask")
    _dev(curve_T, torch.float64, "curve_T")
    _dev(curve_e, torch.float64, "curve_e")
    H, W = _hw(t)
    nby, nbx = -(-H // lb_h), -(-W // lb_w)
    dev = t.device
    T = torch.empty((nby, nbx), dtype=torch.float32, device=dev)
    eb = torch.empty((nby, nbx), dtype=torch.float64, device=dev)
    nb = torch.empty((nby, nbx), dtype=torch.int32, device=dev)
    ws = _ws(lib().mpr_calibrate_workspace_bytes(H, W, lb_h, lb_w), dev)
    _check(lib().mpr_calibrate_temperature(_p(t), _p(mask), H, W, lb_h, lb_w, q, J, _p(curve_T), _p(curve_e),
                                           int(curve_T.numel()), _p(T), _p(eb), _p(nb), _p(ws), ws.numel(),
                                           _stream()))
    return T, eb, nb


def mpr_calibrate_temperature_noalloc(t, mask, lb_h, lb_w, curve_T, curve_e, q=0.5, J=1.0, out=None):
    """mpr_calibrate_temperature with the library's static device scratch instead of a workspace.  `out` = (T, e_b,
    n_b) preallocated outputs ([nby, nbx] float32, float64, int32) makes the call allocate nothing at all."""
    _dev(t, torch.float32, "t")
    _dev(mask, torch.uint8, "mask")
    _dev(curve_T, torch.float64, "curve_T")
    _dev(curve_e, torch.float64, "curve_e")
    H, W = _hw(t)
    nby, nbx = -(-H // lb_h), -(-W // lb_w)
    if out is None:
        out = (torch.empty((nby, nbx), dtype=torch.float32, device=t.device),
               torch.empty((nby, nbx), dtype=torch.float64, device=t.device),
               torch.empty((nby, nbx), dtype=torch.int32, device=t.device))
    T, eb, nb = out
    for x, dt, name in ((T, torch.float32, "T"), (eb, torch.float64, "e_b"), (nb, torch.int32, "n_b")):
        _dev(x, dt, name)
        if x.numel() != nby * nbx:
            raise ValueError(f"{name} has {x.numel()} entries, the grid has {nby * nbx} blocks")
    _check(lib().mpr_calibrate_temperature_noalloc(_p(t), _p(mask), H, W, lb_h, lb_w, q, J, _p(curve_T),
                                                   _p(curve_e), int(curve_T.numel()), _p(T), _p(eb), _p(nb),
                                                   _stream()))
    return T, eb, nb


def mpr_calibrate_directional(t, mask, lb_h, lb_w, curve_T, curve_e, q=0.5, J=1.0):
    """Per-block temperatures of the horizontal and of the vertical sample bonds, (Tx, Ty) each [nby, nbx]."""
    _dev(t, torch.float32, "t")
    _dev(mask, torch.uint8, "mask")
    _dev(curve_T, torch.float64, "curve_T")
    _dev(curve_e, torch.float64, "curve_e")
    H, W = _hw(t)
    nby, nbx = -(-H // lb_h), -(-W // lb_w)
    dev = t.device
    Tx = torch.empty((nby, nbx), dtype=torch.float32, device=dev)
    Ty = torch.empty((nby, nbx), dtype=torch.float32, device=dev)
    ws = _ws(lib().mpr_calibrate_workspace_bytes(H, W, lb_h, lb_w), dev)
    _check(lib().mpr_calibrate_directional(_p(t), _p(mask), H, W, lb_h, lb_w, q, J, _p(curve_T), _p(curve_e),
                                           int(curve_T.numel()), _p(Tx), _p(Ty), _p(ws), ws.numel(), _stream()))
    return Tx, Ty


@dataclass
class SimOutput:
    state: torch.Tensor        # [R, H, W] float32
    acc: torch.Tensor          # [H, W] float64
    energy: torch.Tensor       # [k* + 1] float64 (empty if not requested)
    sweeps: int                # k*
    converged: bool


def mpr_simulate(t, mask, T_blocks, lb_h, lb_w, cfg: SimConfig, state=None, want_energy=True,
                 workspace: torch.Tensor | None = None) -> SimOutput:
    _dev(t, torch.float32, "t")
    _dev(mask, torch.uint8, "mask")
    _dev(T_blocks, torch.float32, "T_blocks")
    H, W = _hw(t)
    _check_T(T_blocks, H, W, lb_h, lb_w, cfg)
    dev = t.device
    c = cfg.to_c()
    if state is None:
        state = torch.empty((cfg.n_real, H, W), dtype=torch.float32, device=dev)
    else:
        _dev(state, torch.float32, "state")
        if tuple(state.shape) != (cfg.n_real, H, W):
            raise ValueError("state must be [n_real, H, W]")
    acc = torch.empty((H, W), dtype=torch.float64, device=dev)
    cap = (cfg.n_max if cfg.stop_mode != STOP_FIXED else cfg.n_eq) + 1
    energy = torch.empty(cap, dtype=torch.float64, device=dev) if want_energy else None
    need = lib().mpr_simulate_workspace_bytes(H, W, lb_h, lb_w, ctypes.byref(c))
    ws = workspace if workspace is not None and workspace.numel() >= need else _ws(need, dev)
    k = _i32(0)
    st = _check(lib().mpr_simulate(_p(t), _p(mask), H, W, _p(T_blocks), lb_h, lb_w, ctypes.byref(c), _p(state),
                                   _p(acc), _p(energy), ctypes.byref(k), _p(ws), ws.numel(), _stream()),
                allow_warn=True)
    ks = int(k.value)
    en = energy[: ks + 1] if energy is not None else torch.empty(0, dtype=torch.float64, device=dev)
    return SimOutput(state=state, acc=acc, energy=en, sweeps=ks, converged=(st == MPR_OK))


def _dhw(x):
    if x.dim() != 3:
        raise ValueError("expected a [D, H, W] tensor")
    return int(x.shape[0]), int(x.shape[1]), int(x.shape[2])


def _blocks3(D, H, W, lb_d, lb_h, lb_w):
    return -(-D // lb_d), -(-H // lb_h), -(-W // lb_w)


def mpr_reference_curve3d(T_grid: torch.Tensor, L: int = 32, n_therm: int = 500, n_meas: int = 1000, seed: int = 0,
                          q: float = 0.5):
    """Matching curve of the cubic lattice: equilibrium energy per bond on a periodic L^3 lattice per temperature."""
    _dev(T_grid, torch.float32, "T_grid")
    nT = int(T_grid.numel())
    e = torch.empty(nT, dtype=torch.float64, device=T_grid.device)
    ws = _ws(lib().mpr_reference_curve3d_workspace_bytes(nT, L), T_grid.device)
    _check(lib().mpr_reference_curve3d(q, _p(T_grid), nT, L, n_therm, n_meas, seed, _p(e), _p(ws), ws.numel(),
                                       _stream()))
    return e


def mpr_calibrate_temperature3d(t, mask, lb_d, lb_h, lb_w, curve_T, curve_e, q=0.5, J=1.0):
    """Per-3D-block temperatures (T, e_b, n_b), each [nbz, nby, nbx]."""
    _dev(t, torch.float32, "t")
    _dev(mask, torch.uint8, "mask")
    _dev(curve_T, torch.float64, "curve_T")
    _dev(curve_e, torch.float64, "curve_e")
    D, H, W = _dhw(t)
    shp = _blocks3(D, H, W, lb_d, lb_h, lb_w)
    dev = t.device
    T = torch.empty(shp, dtype=torch.float32, device=dev)
    eb = torch.empty(shp, dtype=torch.float64, device=dev)
    nb = torch.empty(shp, dtype=torch.int32, device=dev)
    ws = _ws(lib().mpr_calibrate3d_workspace_bytes(D, H, W, lb_d, lb_h, lb_w), dev)
    _check(lib().mpr_calibrate_temperature3d(_p(t), _p(mask), D, H, W, lb_d, lb_h, lb_w, q, J, _p(curve_T),
                                             _p(curve_e), int(curve_T.numel()), _p(T), _p(eb), _p(nb), _p(ws),
                                             ws.numel(), _stream()))
    return T, eb, nb


def mpr_simulate3d(t, mask, T_blocks, lb_d, lb_h, lb_w, cfg: SimConfig, state=None, want_energy=True,
                   workspace: torch.Tensor | None = None) -> SimOutput:
    """Conditional simulation of a [D, H, W] scene; state [n_real, D, H, W], acc [D, H, W]."""
    _dev(t, torch.float32, "t")
    _dev(mask, torch.uint8, "mask")
    _dev(T_blocks, torch.float32, "T_blocks")
    D, H, W = _dhw(t)
    nb = _blocks3(D, H, W, lb_d, lb_h, lb_w)
    if T_blocks.numel() != nb[0] * nb[1] * nb[2]:
        raise ValueError(f"T_blocks has {T_blocks.numel()} entries, the grid has {nb[0] * nb[1] * nb[2]} blocks")
    dev = t.device
    c = cfg.to_c()
    if state is None:
        state = torch.empty((cfg.n_real, D, H, W), dtype=torch.float32, device=dev)
    else:
        _dev(state, torch.float32, "state")
        if tuple(state.shape) != (cfg.n_real, D, H, W):
            raise ValueError("state must be [n_real, D, H, W]")
    acc = torch.empty((D, H, W), dtype=torch.float64, device=dev)
    cap = (cfg.n_max if cfg.stop_mode != STOP_FIXED else cfg.n_eq) + 1
    energy = torch.empty(cap, dtype=torch.float64, device=dev) if want_energy else None
    need = lib().mpr_simulate3d_workspace_bytes(D, H, W, lb_d, lb_h, lb_w, ctypes.byref(c))
    ws = workspace if workspace is not None and workspace.numel() >= need else _ws(need, dev)
    k = _i32(0)
    st = _check(lib().mpr_simulate3d(_p(t), _p(mask), D, H, W, _p(T_blocks), lb_d, lb_h, lb_w, ctypes.byref(c),
                                     _p(state), _p(acc), _p(energy), ctypes.byref(k), _p(ws), ws.numel(), _stream()),
                allow_warn=True)
    ks = int(k.value)
    en = energy[: ks + 1] if energy is not None else torch.empty(0, dtype=torch.float64, device=dev)
    return SimOutput(state=state, acc=acc, energy=en, sweeps=ks, converged=(st == MPR_OK))


def mpr_sweep(state, mask, T_blocks, lb_h, lb_w, cfg: SimConfig, k_first: int, n_sweeps: int, want_energy=False,
              state_alt: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Continue the chains in `state` [n_real, H, W] with sweeps k_first .. k_first + n_sweeps - 1.  The kernels
    alternate between `state` and `state_alt` (a copy of `state` is made when it is not given); the result is
    copied back into `state` when it ends in `state_alt`.  Returns the energies after each sweep (or None)."""
    _dev(state, torch.float32, "state")
    _dev(mask, torch.uint8, "mask")
    _dev(T_blocks, torch.float32, "T_blocks")
    H, W = _hw(mask)
    _check_T(T_blocks, H, W, lb_h, lb_w, cfg)
    if tuple(state.shape) != (cfg.n_real, H, W):
        raise ValueError("state must be [n_real, H, W]")
    if state_alt is None:
        state_alt = state.clone()
    else:
        _dev(state_alt, torch.float32, "state_alt")
        if state_alt.shape != state.shape:
            raise ValueError("state_alt must have the shape of state")
    c = cfg.to_c()
    energy = torch.empty(max(n_sweeps, 1), dtype=torch.float64, device=state.device) if want_energy else None
    need = lib().mpr_sweep_workspace_bytes(H, W, lb_h, lb_w, ctypes.byref(c))
    ws = workspace if workspace is not None and workspace.numel() >= need else _ws(need, state.device)
    _check(lib().mpr_sweep(_p(state), _p(state_alt), _p(mask), H, W, _p(T_blocks), lb_h, lb_w, ctypes.byref(c),
                           int(k_first), int(n_sweeps), _p(energy), _p(ws), ws.numel(), _stream()))
    if n_sweeps % 2 == 1:
        state.copy_(state_alt)
    return energy[:n_sweeps] if energy is not None else None


def mpr_predict(acc, z, mask, n_samples, rng):
    _dev(acc, torch.float64, "acc")
    _dev(z, torch.float32, "z")
    _dev(mask, torch.uint8, "mask")
    _dev(rng, torch.float64, "range")
    H, W = _hw(z)
    zhat = torch.empty_like(z)
    _check(lib().mpr_predict(_p(acc), _p(z), _p(mask), H, W, int(n_samples), _p(rng), _p(zhat), _stream()))
    return zhat


def mpr_validate(zhat, truth, eval_mask):
    _dev(zhat, torch.float32, "zhat")
    _dev(truth, torch.float32, "truth")
    _dev(eval_mask, torch.uint8, "eval_mask")
    n = int(zhat.numel())
    out = torch.empty(2, dtype=torch.float64, device=zhat.device)
    ws = _ws(lib().mpr_validate_workspace_bytes(n), zhat.device)
    _check(lib().mpr_validate(_p(zhat), _p(truth), _p(eval_mask), n, _p(out), _p(ws), ws.numel(), _stream()))
    return out


def mpr_sst_temperatures(T_blocks, H: int, W: int, lb_h: int, lb_w: int, r_s: int = 1, n_s: int = 5):
    """Sec. 2.2.3: site temperatures [H, W] float32 from the block map (n_s passes of the radius-r_s window mean)."""
    _dev(T_blocks, torch.float32, "T_blocks")
    if T_blocks.numel() != ((H + lb_h - 1) // lb_h) * ((W + lb_w - 1) // lb_w):
        raise ValueError("T_blocks must hold one temperature per lb_h x lb_w block")
    dev = T_blocks.device
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    ws = _ws(lib().mpr_sst_temperatures_workspace_bytes(H, W), dev)
    _check(lib().mpr_sst_temperatures(_p(T_blocks), H, W, lb_h, lb_w, r_s, n_s, _p(out), _p(ws), ws.numel(),
                                      _stream()))
    return out


PROBE_NAMES = ("v_add_u32", "v_mad_u64_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_bitop3_b32", "v_sin_f32", "v_cos_f32",
               "v_exp_f32", "v_cvt_f32_u32", "v_xor_b32", "v_mad_u64_u32+v_add_u32", "v_mad_u64_u32+v_bitop3_b32")


def mpr_probe_instruction_rates(device=None):
    """Issue cost of each probed instruction relative to v_add_u32 (dict name -> cost) and the device time per
    wave-instruction of v_add_u32 in ns."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    ws = _ws(lib().mpr_probe_instruction_rates_workspace_bytes(), dev)
    cost = (ctypes.c_double * len(PROBE_NAMES))()
    add_ns = ctypes.c_double(0.0)
    _check(lib().mpr_probe_instruction_rates(cost, len(PROBE_NAMES), ctypes.byref(add_ns), _p(ws), ws.numel(),
                                             _stream()))
    return {n: float(c) for n, c in zip(PROBE_NAMES, cost)}, float(add_ns.value)


def mpr_block_energy(state, mask, lb_h, lb_w, q=0.5, J=1.0):
    """H_b per realization: [R, nby * nbx] float64."""
    _dev(state, torch.float32, "state")
    _dev(mask, torch.uint8, "mask")
    H, W = _hw(mask)
    R = int(state.shape[0])
    if tuple(state.shape) != (R, H, W):
        raise ValueError("state must be [R, H, W]")
    B = (-(-H // lb_h)) * (-(-W // lb_w))
    out = torch.empty((R, B), dtype=torch.float64, device=state.device)
    ws = _ws(lib().mpr_block_energy_workspace_bytes(H, W, lb_h, lb_w, R), state.device)
    _check(lib().mpr_block_energy(_p(state), _p(mask), H, W, lb_h, lb_w, q, J, R, _p(out), _p(ws), ws.numel(),
                                  _stream()))
    return out


def mpr_temperature_grad(state, H_blocks, grad_zhat, mask, rng, T_blocks):
    """dL/dT_b [B] float64 from the final states of a run with one sampling sweep."""
    _dev(state, torch.float32, "state")
    _dev(H_blocks, torch.float64, "H_blocks")
    _dev(grad_zhat, torch.float32, "grad_zhat")
    _dev(mask, torch.uint8, "mask")
    _dev(rng, torch.float64, "range")
    _dev(T_blocks, torch.float32, "T_blocks")
    H, W = _hw(mask)
    R = int(state.shape[0])
    B = int(H_blocks.shape[1])
    if T_blocks.numel() != B or tuple(H_blocks.shape) != (R, B):
        raise ValueError("H_blocks must be [R, B] and T_blocks must have B entries")
    dT = torch.empty(B, dtype=torch.float64, device=state.device)
    ws = _ws(lib().mpr_temperature_grad_workspace_bytes(H, W, R), state.device)
    _check(lib().mpr_temperature_grad(_p(state), _p(H_blocks), _p(grad_zhat), _p(mask), H, W, R, B, _p(rng),
                                      _p(T_blocks), _p(dT), _p(ws), ws.numel(), _stream()))
    return dT


@dataclass
class BatchOutput:
    outputs: list              # SimOutput per scene
    tile_h: int                # tile height the sweep kernel used
    converged: bool


def mpr_simulate_batched(scenes, cfg: SimConfig, tile_h: int = 0, want_energy: bool = False,
                         workspace: torch.Tensor | None = None) -> BatchOutput:
    """scenes: list of dicts with t [H, W] f32, mask [H, W] u8, T_blocks f32, block (lb_h, lb_w), scene_id.
    One batched call; every scene's result equals mpr_simulate with its own scene_id."""
    n = len(scenes)
    arr = (mpr_scene * n)()
    outs = []
    cap = (cfg.n_max if cfg.stop_mode != STOP_FIXED else cfg.n_eq) + 1
    for i, sc in enumerate(scenes):
        t, mask, T = sc["t"], sc["mask"], sc["T_blocks"]
        _dev(t, torch.float32, "t")
        _dev(mask, torch.uint8, "mask")
        _dev(T, torch.float32, "T_blocks")
        H, W = _hw(t)
        lb_h, lb_w = sc["block"]
        _check_T(T, int(t.shape[-2]), int(t.shape[-1]), int(lb_h), int(lb_w), cfg)
        state = torch.empty((cfg.n_real, H, W), dtype=torch.float32, device=t.device)
        acc = torch.empty((H, W), dtype=torch.float64, device=t.device)
        en = torch.empty(cap, dtype=torch.float64, device=t.device) if want_energy else None
        arr[i] = mpr_scene(H, W, lb_h, lb_w, int(sc.get("scene_id", i)), t.data_ptr(), mask.data_ptr(), T.data_ptr(),
                           state.data_ptr(), acc.data_ptr(), en.data_ptr() if en is not None else None)
        outs.append((state, acc, en))
    c = cfg.to_c()
    need = lib().mpr_simulate_batched_workspace_bytes(arr, n, ctypes.byref(c))
    dev = scenes[0]["t"].device
    ws = workspace if workspace is not None and workspace.numel() >= need else _ws(need, dev)
    done = (_i32 * n)()
    conv = (_i32 * n)()
    used = _i32(0)
    st = _check(lib().mpr_simulate_batched(arr, n, ctypes.byref(c), int(tile_h), done, conv, ctypes.byref(used),
                                           _p(ws), ws.numel(), _stream()), allow_warn=True)
    res = []
    for i, (state, acc, en) in enumerate(outs):
        k = int(done[i])
        e = en[: k + 1] if en is not None else torch.empty(0, dtype=torch.float64, device=dev)
        res.append(SimOutput(state=state, acc=acc, energy=e, sweeps=k, converged=bool(conv[i])))
    return BatchOutput(outputs=res, tile_h=int(used.value), converged=(st == MPR_OK))
