"""ORACLE — test infrastructure only.

A plain, slow FP64 CPU implementation of the SV-MPR conditional Monte Carlo method (arXiv 2212.01317), written
from the paper.  The arithmetic lives in ``mpr_oracle.c`` (built with gcc, no fast-math); this module loads it
with ctypes and adds numpy-level drivers.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it.  It shares no code with the HIP library ``paper_2212_01317_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")
# the same source built with OpenMP over the realizations of orc_simulate (CPU-baseline timing on all host cores;
# its results equal the single-threaded build's bit for bit)
_LIB_OMP_PATH = os.path.join(_HERE, "liborc_omp.so")

_lib = None
_lib_omp = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, IEEE semantics: no fast-math), single-threaded and with OpenMP."""
    for path, extra in ((_LIB_PATH, []), (_LIB_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", *extra, "-o", tmp,
                                   _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB_PATH


def lib(parallel: bool = False) -> ctypes.CDLL:
    """The oracle library; parallel=True loads the OpenMP build (same results, realizations over threads)."""
    global _lib, _lib_omp
    if parallel:
        if _lib_omp is None:
            if not os.path.exists(_LIB_OMP_PATH):
                build(force=False)
            _lib_omp = ctypes.CDLL(_LIB_OMP_PATH)
            _declare(_lib_omp)
        return _lib_omp
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


def threads(parallel: bool = False) -> int:
    """Threads orc_simulate's realization loops use in the chosen build."""
    return int(lib(parallel).orc_threads())


_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_flt = ctypes.c_float
_dbl = ctypes.c_double


def _declare(L: ctypes.CDLL) -> None:
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_philox4x32_10.restype = None
    L.orc_site_uniforms.argtypes = [_u64, _u32, _u32, _u32, _u32, _i64, _i64, _i64, _f64p]
    L.orc_site_uniforms.restype = None
    L.orc_map_angles.argtypes = [_f32p, _u8p, _i64, _i64, _f32p, _f64p]
    L.orc_map_angles.restype = ctypes.c_int
    L.orc_bond_energy.argtypes = [_flt, _flt, _flt, _flt]
    L.orc_bond_energy.restype = _dbl
    L.orc_block_stats.argtypes = [_f32p, _u8p, _i64, _i64, _i32, _i32, _flt, _flt, _f64p, _i32p, _f64p, _i32p]
    L.orc_block_stats.restype = None
    L.orc_curve_inverse.argtypes = [_dbl, _f64p, _f64p, _i32]
    L.orc_curve_inverse.restype = _dbl
    L.orc_calibrate_blocks.argtypes = [_f64p, _i32p, _i64, _flt, _f64p, _f64p, _i32, _f32p]
    L.orc_calibrate_blocks.restype = ctypes.c_int
    L.orc_sweep.argtypes = [_f32p, _u8p, _i64, _i64, _f32p, _i32, _i32, _flt, _flt, _u64, _u32, _u32, _u32]
    L.orc_sweep.restype = None
    L.orc_energy.argtypes = [_f32p, _i64, _i64, _flt, _flt]
    L.orc_energy.restype = _dbl
    L.orc_reference_curve.argtypes = [_flt, _f32p, _i32, _i32, _i32, _i32, _u64, _f64p]
    L.orc_reference_curve.restype = None
    L.orc_unconditional_sample.argtypes = [_flt, _flt, _i32, _i32, _u64, _u32, _f32p]
    L.orc_unconditional_sample.restype = None
    L.orc_ols_slope.argtypes = [_f64p, _i32]
    L.orc_ols_slope.restype = _dbl
    L.orc_stop_check.argtypes = [_f64p, _i32, _i32, _i32]
    L.orc_stop_check.restype = ctypes.c_int
    L.orc_stop_check_chains.argtypes = [_f64p, _i32, _i32, _i32, _i32, _u8p]
    L.orc_stop_check_chains.restype = ctypes.c_int
    L.orc_simulate.argtypes = [_f32p, _u8p, _i64, _i64, _f32p, _i32, _i32, _flt, _flt, _i32, _i32, _i32, _i32,
                               _i32, _i32, _i32, _i32, _i32, _u64, _u32, _i32, _i32, _i32, _f32p, _f64p, _f64p,
                               ctypes.POINTER(_i32)]
    L.orc_block_stats_directional.argtypes = [_f32p, _u8p, _i64, _i64, _i32, _i32, _flt, _flt, _f64p, _i32p, _f64p,
                                              _i32p]
    L.orc_block_stats_directional.restype = None
    L.orc_sweep_directional.argtypes = [_f32p, _u8p, _i64, _i64, _f32p, _i32, _i32, _flt, _flt, _u64, _u32, _u32,
                                        _u32]
    L.orc_sweep_directional.restype = None
    L.orc_simulate.restype = _i32
    L.orc_sst_temperatures.argtypes = [_f32p, _i64, _i64, _i32, _i32, _i32, _i32, _f32p]
    L.orc_sst_temperatures.restype = None
    L.orc_predict.argtypes = [_f64p, _f32p, _u8p, _i64, _i64, _i64, _f64p, _f32p]
    L.orc_predict.restype = None
    L.orc_validate.argtypes = [_f32p, _f32p, _u8p, _i64, _f64p]
    L.orc_validate.restype = None
    L.orc_block_energy.argtypes = [_f32p, _u8p, _i64, _i64, _i32, _i32, _flt, _flt, _f64p]
    L.orc_block_energy.restype = None
    L.orc_temperature_grad.argtypes = [_f32p, _f64p, _f64p, _i64, _i32, _i64, _f32p, _f64p]
    L.orc_temperature_grad.restype = None
    L.orc_threads.argtypes = []
    L.orc_threads.restype = ctypes.c_int
    # the 3D lattice
    L.orc_site_uniforms3.argtypes = [_u64, _u32, _u32, _u32, _u32, _i64, _i64, _i64, _i64, _i64, _f64p]
    L.orc_site_uniforms3.restype = None
    L.orc_block_stats3.argtypes = [_f32p, _u8p, _i64, _i64, _i64, _i32, _i32, _i32, _flt, _flt, _f64p, _i32p, _f64p,
                                   _i32p]
    L.orc_block_stats3.restype = None
    L.orc_sweep3.argtypes = [_f32p, _u8p, _i64, _i64, _i64, _f32p, _i32, _i32, _i32, _flt, _flt, _u64, _u32, _u32,
                             _u32]
    L.orc_sweep3.restype = None
    L.orc_energy3.argtypes = [_f32p, _i64, _i64, _i64, _flt, _flt]
    L.orc_energy3.restype = _dbl
    L.orc_reference_curve3.argtypes = [_flt, _f32p, _i32, _i32, _i32, _i32, _u64, _f64p]
    L.orc_reference_curve3.restype = None
    L.orc_simulate3.argtypes = [_f32p, _u8p, _i64, _i64, _i64, _f32p, _i32, _i32, _i32, _flt, _flt, _i32, _i32, _i32,
                                _i32, _i32, _i32, _i32, _i32, _i32, _u64, _u32, _f32p, _f64p, _f64p,
                                ctypes.POINTER(_i32)]
    L.orc_simulate3.restype = _i32


# ---------------------------------------------------------------------------------------------------------------
# thin numpy-facing wrappers
# ---------------------------------------------------------------------------------------------------------------

def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def philox4x32_10(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_c(ctr, np.uint32), _c(key, np.uint32), out)
    return out


def site_uniforms(seed, scene, tag, sweep, real, W, x, y):
    out = np.zeros(2, np.float64)
    lib().orc_site_uniforms(seed, scene, tag, sweep, real, W, x, y, out)
    return out


def map_angles(z, mask):
    z = _c(z, np.float32)
    mask = _c(mask, np.uint8)
    H, W = z.shape
    t = np.zeros_like(z)
    rng = np.zeros(2, np.float64)
    rc = lib().orc_map_angles(z, mask, H, W, t, rng)
    if rc != 0:
        raise ValueError({-1: "no observed site", -2: "non-finite observed value"}[rc])
    return t, rng


def bond_energy(ta, tb, q=0.5, J=1.0) -> float:
    return lib().orc_bond_energy(ta, tb, q, J)


def n_blocks(H, W, lb_h, lb_w):
    return (-(-H // lb_h)), (-(-W // lb_w))


def block_stats(t, mask, lb_h, lb_w, q=0.5, J=1.0):
    t = _c(t, np.float32)
    mask = _c(mask, np.uint8)
    H, W = t.shape
    nby, nbx = n_blocks(H, W, lb_h, lb_w)
    B = nby * nbx
    S = np.zeros(B, np.float64)
    N = np.zeros(B, np.int32)
    Ts = np.zeros(B, np.float64)
    No = np.zeros(B, np.int32)
    lib().orc_block_stats(t, mask, H, W, lb_h, lb_w, q, J, S, N, Ts, No)
    return S, N, Ts, No


def block_stats_directional(t, mask, lb_h, lb_w, q=0.5, J=1.0):
    """Eq. (2) per block split by bond direction: (Sh, Nh) horizontal bonds, (Sv, Nv) vertical bonds."""
    t = _c(t, np.float32)
    mask = _c(mask, np.uint8)
    H, W = t.shape
    nby, nbx = n_blocks(H, W, lb_h, lb_w)
    B = nby * nbx
    Sh, Sv = np.zeros(B, np.float64), np.zeros(B, np.float64)
    Nh, Nv = np.zeros(B, np.int32), np.zeros(B, np.int32)
    lib().orc_block_stats_directional(t, mask, H, W, lb_h, lb_w, q, J, Sh, Nh, Sv, Nv)
    return Sh, Nh, Sv, Nv


# Directional coupling: the lowest temperature a direction may take, in units of J (keeps both temperatures > 0, so
# the ratio of the two couplings is finite).
T_MIN_DIRECTIONAL = 1e-3


def calibrate_directional(t, mask, lb_h, lb_w, curve_T, curve_e, q=0.5, J=1.0):
    """Directional coupling (the extension suggested in Sec. 4): each block gets Tx from its horizontal sample bonds
    and Ty from its vertical ones, each by the energy matching and median fill of Sec. 2.2.2 with the (isotropic)
    matching curve, then raised to at least fl32(T_MIN_DIRECTIONAL * J).  Returns (Tx, Ty) as [nby, nbx] float32."""
    H, W = np.shape(t)
    Sh, Nh, Sv, Nv = block_stats_directional(t, mask, lb_h, lb_w, q, J)
    floor = np.float32(T_MIN_DIRECTIONAL * float(J))
    Tx = np.maximum(calibrate_blocks(Sh, Nh, curve_T, curve_e, J), floor)
    Ty = np.maximum(calibrate_blocks(Sv, Nv, curve_T, curve_e, J), floor)
    nby, nbx = n_blocks(H, W, lb_h, lb_w)
    return Tx.reshape(nby, nbx), Ty.reshape(nby, nbx)


def sweep_directional(state, mask, Tx, Ty, lb_h, lb_w, k, q=0.5, J=1.0, seed=0, scene=0, real=0):
    assert state.dtype == np.float32 and state.flags["C_CONTIGUOUS"]
    H, W = state.shape
    T = np.concatenate([_c(Tx, np.float32).ravel(), _c(Ty, np.float32).ravel()])
    lib().orc_sweep_directional(state, _c(mask, np.uint8), H, W, T, lb_h, lb_w, q, J, seed, scene, real, k)


def curve_inverse(e, curve_T, curve_e) -> float:
    cT = _c(curve_T, np.float64)
    ce = _c(curve_e, np.float64)
    return lib().orc_curve_inverse(float(e), cT, ce, len(cT))


def calibrate_blocks(S, N, curve_T, curve_e, J=1.0):
    S = _c(S, np.float64)
    N = _c(N, np.int32)
    cT = _c(curve_T, np.float64)
    ce = _c(curve_e, np.float64)
    T = np.zeros(len(S), np.float32)
    rc = lib().orc_calibrate_blocks(S, N, len(S), J, cT, ce, len(cT), T)
    if rc != 0:
        raise ValueError("no sample bonds")
    return T


def calibrate_temperature(t, mask, lb_h, lb_w, curve_T, curve_e, q=0.5, J=1.0):
    """Eq. (2) per block followed by energy matching and the median fill (Sec. 2.2.2)."""
    H, W = np.shape(t)
    S, N, _, _ = block_stats(t, mask, lb_h, lb_w, q, J)
    T = calibrate_blocks(S, N, curve_T, curve_e, J)
    nby, nbx = n_blocks(H, W, lb_h, lb_w)
    return T.reshape(nby, nbx), S.reshape(nby, nbx), N.reshape(nby, nbx)


def sweep(state, mask, T_blocks, lb_h, lb_w, k, q=0.5, J=1.0, seed=0, scene=0, real=0):
    assert state.dtype == np.float32 and state.flags["C_CONTIGUOUS"]
    H, W = state.shape
    lib().orc_sweep(state, _c(mask, np.uint8), H, W, _c(T_blocks, np.float32).ravel(), lb_h, lb_w, q, J, seed,
                    scene, real, k)


def energy(state, q=0.5, J=1.0) -> float:
    s = _c(state, np.float32)
    H, W = s.shape
    return lib().orc_energy(s, H, W, q, J)


def reference_curve(T_grid, L=64, n_therm=200, n_meas=400, seed=0, q=0.5):
    Tg = _c(T_grid, np.float32)
    e = np.zeros(len(Tg), np.float64)
    lib().orc_reference_curve(q, Tg, len(Tg), L, n_therm, n_meas, seed, e)
    return e


def unconditional_sample(T, L=64, n_sweeps=300, seed=0, chain=0, q=0.5):
    out = np.zeros((L, L), np.float32)
    lib().orc_unconditional_sample(q, T, L, n_sweeps, seed, chain, out)
    return out


def ols_slope(y) -> float:
    y = _c(y, np.float64)
    return lib().orc_ols_slope(y, len(y))


def stop_check(e, k, n_fit=20, n_f=5) -> bool:
    return bool(lib().orc_stop_check(_c(e, np.float64), k, n_fit, n_f))


def stop_check_chains(ser, k, passed, n_fit=20, n_f=5) -> bool:
    """Per-chain test at sweep k: ser[j, r] is chain r's energy after sweep j (j = 0 .. k); `passed` (uint8 [R])
    holds the chains that have passed and is updated in place."""
    ser = _c(ser, np.float64)
    assert passed.dtype == np.uint8 and passed.flags["C_CONTIGUOUS"] and passed.size == ser.shape[1]
    return bool(lib().orc_stop_check_chains(ser, ser.shape[1], k, n_fit, n_f, passed))


@dataclass
class SimConfig:
    q: float = 0.5
    J: float = 1.0
    n_real: int = 1
    real_offset: int = 0
    init_mode: int = 1          # 0 random start (MPR), 1 block-mean start (SV-MPR)
    stop_mode: int = 0          # 0 fixed n_eq, 1 automatic equilibrium test, 2 the same per chain
    n_eq: int = 50
    n_samp: int = 1
    n_fit: int = 20
    n_f: int = 5
    n_max: int = 1000
    seed: int = 0
    scene: int = 0
    t_mode: int = 0             # 0 block temperatures (BST), 1 one temperature per site (SST)
    order: int = 0              # 0 single checkerboard, 1 double checkerboard over the blocks
    directional: int = 0        # 1: T_blocks holds Tx of every block, then Ty (directional coupling, SC order)


@dataclass
class SimResult:
    state: np.ndarray
    acc: np.ndarray
    energy: np.ndarray
    k_star: int
    converged: bool


def simulate(t, mask, T_blocks, lb_h, lb_w, cfg: SimConfig, parallel: bool = False) -> SimResult:
    t = _c(t, np.float32)
    mask = _c(mask, np.uint8)
    H, W = t.shape
    R = cfg.n_real
    state = np.zeros((R, H, W), np.float32)
    acc = np.zeros((H, W), np.float64)
    ncap = (cfg.n_max if cfg.stop_mode != 0 else cfg.n_eq) + 1
    en = np.zeros(ncap, np.float64)
    conv = _i32(0)
    k = lib(parallel).orc_simulate(t, mask, H, W, _c(T_blocks, np.float32).ravel(), lb_h, lb_w, cfg.q, cfg.J, R,
                           cfg.real_offset, cfg.init_mode, cfg.stop_mode, cfg.n_eq, cfg.n_samp, cfg.n_fit, cfg.n_f,
                           cfg.n_max, cfg.seed, cfg.scene, cfg.t_mode, cfg.order, cfg.directional, state, acc, en,
                           ctypes.byref(conv))
    return SimResult(state=state, acc=acc, energy=en[: k + 1].copy(), k_star=int(k), converged=bool(conv.value))


def sst_temperatures(T_blocks, H, W, lb_h, lb_w, r_s=1, n_s=5):
    """Sec. 2.2.3: site-specific temperatures [H, W] float32 from the block map by n_s passes of the radius-r_s
    window mean (orc_sst_temperatures)."""
    out = np.zeros((H, W), np.float32)
    lib().orc_sst_temperatures(_c(T_blocks, np.float32).ravel(), H, W, lb_h, lb_w, r_s, n_s, out)
    return out


def predict(acc, z, mask, n_samples, rng):
    acc = _c(acc, np.float64)
    z = _c(z, np.float32)
    H, W = z.shape
    zhat = np.zeros_like(z)
    lib().orc_predict(acc, z, _c(mask, np.uint8), H, W, n_samples, _c(rng, np.float64), zhat)
    return zhat


def validate(zhat, truth, eval_mask):
    out = np.zeros(2, np.float64)
    zh = _c(zhat, np.float32).ravel()
    lib().orc_validate(zh, _c(truth, np.float32).ravel(), _c(eval_mask, np.uint8).ravel(), zh.size, out)
    return float(out[0]), float(out[1])


def run_pipeline(z, mask, lb_h, lb_w, curve_T, curve_e, cfg: SimConfig):
    """Sec. 2: map -> per-block calibration -> conditional simulation -> conditional-mean prediction."""
    t, rng = map_angles(z, mask)
    T, _, _ = calibrate_temperature(t, mask, lb_h, lb_w, curve_T, curve_e, cfg.q, cfg.J)
    res = simulate(t, mask, T, lb_h, lb_w, cfg)
    zhat = predict(res.acc, z, mask, cfg.n_real * cfg.n_samp, rng)
    return dict(t=t, range=rng, T=T, sim=res, zhat=zhat)


def block_energy(state, mask, lb_h, lb_w, q=0.5, J=1.0):
    """H_b of one state [H, W] (bonds with a gap end; gap-gap bonds across blocks split one half each)."""
    s = _c(state, np.float32)
    H, W = s.shape
    nby, nbx = n_blocks(H, W, lb_h, lb_w)
    out = np.zeros(nby * nbx, np.float64)
    lib().orc_block_energy(s, _c(mask, np.uint8), H, W, lb_h, lb_w, q, J, out)
    return out


def temperature_grad(states, Hrb, w, T_blocks):
    """Score-function estimate of dL/dT_b from R final states [R, H, W] (one sampling sweep), block energies
    [R, B] and weights w [H, W] = dL/dzhat * (zmax - zmin) at gaps (0 at samples): E[zhat] = zmin + span * E[t]."""
    st = _c(states, np.float32)
    R = st.shape[0]
    HW = st.shape[1] * st.shape[2]
    Hrb = _c(Hrb, np.float64)
    B = Hrb.shape[1]
    out = np.zeros(B, np.float64)
    lib().orc_temperature_grad(st, Hrb, _c(w, np.float64).ravel(), HW, R, B, _c(T_blocks, np.float32).ravel(), out)
    return out


# ---------------------------------------------------------------------------------------------------------------
# the 3D lattice (Sec. 4 extension): grids are [D, H, W], blocks (lb_d, lb_h, lb_w)
# ---------------------------------------------------------------------------------------------------------------

def n_blocks3(D, H, W, lb_d, lb_h, lb_w):
    return (-(-D // lb_d)), (-(-H // lb_h)), (-(-W // lb_w))


def site_uniforms3(seed, scene, tag, sweep, real, H, W, x, y, z):
    out = np.zeros(2, np.float64)
    lib().orc_site_uniforms3(seed, scene, tag, sweep, real, H, W, x, y, z, out)
    return out


def block_stats3(t, mask, lb_d, lb_h, lb_w, q=0.5, J=1.0):
    t = _c(t, np.float32)
    mask = _c(mask, np.uint8)
    D, H, W = t.shape
    B = int(np.prod(n_blocks3(D, H, W, lb_d, lb_h, lb_w)))
    S, Ts = np.zeros(B, np.float64), np.zeros(B, np.float64)
    N, No = np.zeros(B, np.int32), np.zeros(B, np.int32)
    lib().orc_block_stats3(t, mask, D, H, W, lb_d, lb_h, lb_w, q, J, S, N, Ts, No)
    return S, N, Ts, No


def calibrate_temperature3(t, mask, lb_d, lb_h, lb_w, curve_T, curve_e, q=0.5, J=1.0):
    """Eq. (2) per 3D block, energy matching with a matching curve of the 3D model, median fill."""
    D, H, W = np.shape(t)
    S, N, _, _ = block_stats3(t, mask, lb_d, lb_h, lb_w, q, J)
    T = calibrate_blocks(S, N, curve_T, curve_e, J)
    shp = n_blocks3(D, H, W, lb_d, lb_h, lb_w)
    return T.reshape(shp), S.reshape(shp), N.reshape(shp)


def sweep3(state, mask, T_blocks, lb_d, lb_h, lb_w, k, q=0.5, J=1.0, seed=0, scene=0, real=0):
    assert state.dtype == np.float32 and state.flags["C_CONTIGUOUS"]
    D, H, W = state.shape
    lib().orc_sweep3(state, _c(mask, np.uint8), D, H, W, _c(T_blocks, np.float32).ravel(), lb_d, lb_h, lb_w, q, J,
                     seed, scene, real, k)


def energy3(state, q=0.5, J=1.0) -> float:
    s = _c(state, np.float32)
    D, H, W = s.shape
    return lib().orc_energy3(s, D, H, W, q, J)


def reference_curve3(T_grid, L=16, n_therm=200, n_meas=400, seed=0, q=0.5):
    Tg = _c(T_grid, np.float32)
    e = np.zeros(len(Tg), np.float64)
    lib().orc_reference_curve3(q, Tg, len(Tg), L, n_therm, n_meas, seed, e)
    return e


def simulate3(t, mask, T_blocks, lb_d, lb_h, lb_w, cfg: SimConfig, parallel: bool = False) -> SimResult:
    """Conditional simulation of a [D, H, W] scene (block temperatures, single-checkerboard order)."""
    t = _c(t, np.float32)
    mask = _c(mask, np.uint8)
    D, H, W = t.shape
    R = cfg.n_real
    state = np.zeros((R, D, H, W), np.float32)
    acc = np.zeros((D, H, W), np.float64)
    ncap = (cfg.n_max if cfg.stop_mode != 0 else cfg.n_eq) + 1
    en = np.zeros(ncap, np.float64)
    conv = _i32(0)
    k = lib(parallel).orc_simulate3(t, mask, D, H, W, _c(T_blocks, np.float32).ravel(), lb_d, lb_h, lb_w, cfg.q,
                                    cfg.J, R, cfg.real_offset, cfg.init_mode, cfg.stop_mode, cfg.n_eq, cfg.n_samp,
                                    cfg.n_fit, cfg.n_f, cfg.n_max, cfg.seed, cfg.scene, state, acc, en,
                                    ctypes.byref(conv))
    return SimResult(state=state, acc=acc, energy=en[: k + 1].copy(), k_star=int(k), converged=bool(conv.value))
