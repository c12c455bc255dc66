"""The C-ABI library loads and exports every entry point include/mpr.h declares; host-side checks reject bad
arguments before any device work (no GPU needed)."""
import ctypes

import pytest

from paper_2212_01317_amd import _lib


def test_header_symbols_exported():
    L = _lib.lib()
    names = _lib.header_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib._SIGS), "binding signatures and header declarations differ"


def test_abi_version():
    assert _lib.lib().mpr_abi_version() == 10000


def test_workspace_queries_are_host_only():
    L = _lib.lib()
    assert L.mpr_map_workspace_bytes(128, 128) > 0
    assert L.mpr_block_stats_workspace_bytes(4096, 4096, 32, 32) >= 128 * 128 * 24
    assert L.mpr_calibrate_workspace_bytes(1024, 1024, 16, 16) > 0
    assert L.mpr_reference_curve_workspace_bytes(121, 128) >= 121 * 128 * 128 * 4
    cfg = _lib.SimConfig(n_real=256).to_c()
    big = L.mpr_simulate_workspace_bytes(4096, 4096, 32, 32, ctypes.byref(cfg))
    assert big > 0
    cfg2 = _lib.SimConfig(n_real=512).to_c()
    assert L.mpr_simulate_workspace_bytes(4096, 4096, 32, 32, ctypes.byref(cfg2)) > big
    assert L.mpr_validate_workspace_bytes(0) > 0


@pytest.mark.parametrize("H,W", [(0, 5), (5, 0), (-1, 3), (1 << 21, 4)])
def test_bad_shapes_rejected_before_device_work(H, W):
    L = _lib.lib()
    st = L.mpr_map_angles(None, None, H, W, None, None, None, 0, None)
    assert st == 2
    assert b"grid" in L.mpr_last_error()


def test_bad_config_rejected():
    L = _lib.lib()
    dummy = ctypes.c_void_p(0x1000)     # never dereferenced: the checks fail first
    for kw in (dict(q=0.75), dict(J=0.0), dict(n_real=0), dict(init_mode=7), dict(stop_mode=3),
               dict(stop_mode=_lib.STOP_AUTO, n_fit=1), dict(scene_id=1 << 28)):
        cfg = _lib.SimConfig(**kw).to_c()
        st = L.mpr_simulate(dummy, dummy, 8, 8, dummy, 4, 4, ctypes.byref(cfg), dummy, dummy, None, None, dummy,
                            1 << 30, None)
        assert st == 1, kw
    cfg = _lib.SimConfig().to_c()
    st = L.mpr_simulate(dummy, dummy, 8, 8, dummy, 4, 4, ctypes.byref(cfg), dummy, dummy, None, None, dummy, 16, None)
    assert st == 6      # workspace too small
    st = L.mpr_simulate(dummy, dummy, 8, 8, dummy, 0, 4, ctypes.byref(cfg), dummy, dummy, None, None, dummy, 16, None)
    assert st == 2      # bad block


def test_reference_curve_rejects_odd_lattice():
    L = _lib.lib()
    dummy = ctypes.c_void_p(0x1000)
    assert L.mpr_reference_curve(0.5, dummy, 4, 15, 10, 10, 0, dummy, dummy, 1 << 30, None) == 2
    assert L.mpr_reference_curve(0.6, dummy, 4, 16, 10, 10, 0, dummy, dummy, 1 << 30, None) == 1


def test_noalloc_calibration_rejects_sizes_beyond_its_scratch():
    """The entry point without a workspace refuses, before any device work, a grid whose calibration scratch exceeds
    the static array (1 x 1 blocks on 4096^2 need 576 MiB), and accepts the size check of the headline shape."""
    L = _lib.lib()
    dummy = ctypes.c_void_p(0x1000)     # never dereferenced: the size check fails first
    assert L.mpr_calibrate_workspace_bytes(4096, 4096, 1, 1) > 16 << 20
    assert L.mpr_calibrate_workspace_bytes(16384, 16384, 32, 32) <= 16 << 20
    st = L.mpr_calibrate_temperature_noalloc(dummy, dummy, 4096, 4096, 1, 1, 0.5, 1.0, dummy, dummy, 4, dummy, None,
                                             None, None)
    assert st == 6
    assert b"static scratch" in L.mpr_last_error()
    st = L.mpr_calibrate_temperature_noalloc(dummy, dummy, 0, 4096, 32, 32, 0.5, 1.0, dummy, dummy, 4, dummy, None,
                                             None, None)
    assert st == 2


def test_binding_refuses_cpu_tensors():
    import torch
    with pytest.raises(ValueError):
        _lib.mpr_map_angles(torch.zeros(4, 4), torch.ones(4, 4, dtype=torch.uint8))


def test_batched_workspace_follows_the_batch_kernel():
    """Host-only size queries: with 64 realizations (or sweep_kernel = LANES) the batch runs on the persistent lane
    sweep, whose workspace holds two lane-layout state buffers (realizations padded to 64) per scene, added over the
    scenes; with fewer realizations, sweep_kernel = TILES, or scenes whose temperature blocks the lane sweep looks
    up in different ways, the batch runs on the persistent tile kernel."""
    L = _lib.lib()
    auto = _lib.SimConfig(n_real=64).to_c()
    tiles = _lib.SimConfig(n_real=64, sweep_kernel=_lib.SWEEP_TILES).to_c()
    few = _lib.SimConfig(n_real=8).to_c()
    few_tiles = _lib.SimConfig(n_real=8, sweep_kernel=_lib.SWEEP_TILES).to_c()
    few_lanes = _lib.SimConfig(n_real=8, sweep_kernel=_lib.SWEEP_LANES).to_c()
    big, small = (1024, 800), (70, 130)

    def batch(shapes, lb=16):
        arr = (_lib.mpr_scene * len(shapes))()
        for i, sh in enumerate(shapes):
            H, W = sh[:2]
            b = sh[2] if len(sh) > 2 else lb
            arr[i] = _lib.mpr_scene(H, W, b, b, i, None, None, None, None, None, None)
        return arr, len(shapes)

    ws = lambda shapes, cfg: L.mpr_simulate_batched_workspace_bytes(*batch(shapes), ctypes.byref(cfg))
    lane_bufs = lambda H, W: 2 * 64 * H * W * 4
    assert ws([big], auto) >= lane_bufs(*big)
    assert ws([big, small], auto) >= ws([big], auto) + lane_bufs(*small)
    assert ws([big], tiles) != ws([big], auto)
    assert ws([big, small], few) == ws([big, small], few_tiles)
    assert ws([big, small], few_lanes) >= lane_bufs(*big) + lane_bufs(*small)
    # 16-wide blocks take two temperature columns per window, 24-wide ones line up with the bands: tile batch
    assert ws([big, (70, 130, 24)], auto) == ws([big, (70, 130, 24)], tiles)


def test_3d_arguments_rejected_before_device_work():
    """The 3D entry points check shapes, blocks, the configuration and the workspace on the host first."""
    L = _lib.lib()
    dummy = ctypes.c_void_p(0x1000)
    cfg = _lib.SimConfig(n_real=64, stop_mode=_lib.STOP_FIXED, n_eq=2).to_c()
    for D, H, W in ((0, 4, 4), (4, 0, 4), (4, 4, 70000), (65535, 65535, 64)):
        st = L.mpr_simulate3d(dummy, dummy, D, H, W, dummy, 2, 2, 2, ctypes.byref(cfg), dummy, dummy, None, None,
                              dummy, 1 << 40, None)
        assert st == 2, (D, H, W)
    st = L.mpr_simulate3d(dummy, dummy, 4, 4, 4, dummy, 0, 2, 2, ctypes.byref(cfg), dummy, dummy, None, None, dummy,
                          1 << 40, None)
    assert st == 2                                   # a block side below 1
    for kw in (dict(t_mode=_lib.T_SITE), dict(order=_lib.ORDER_DC), dict(coupling=_lib.COUPLING_DIRECTIONAL),
               dict(stop_mode=5), dict(stop_mode=_lib.STOP_AUTO_CHAIN, n_fit=1)):
        c = _lib.SimConfig(n_real=64, **kw).to_c()
        st = L.mpr_simulate3d(dummy, dummy, 4, 4, 4, dummy, 2, 2, 2, ctypes.byref(c), dummy, dummy, None, None, dummy,
                              1 << 40, None)
        assert st == 1, kw
    need = L.mpr_simulate3d_workspace_bytes(4, 4, 4, 2, 2, 2, ctypes.byref(cfg))
    assert need >= 64 * 64 * 4                        # the lane copy of the state
    st = L.mpr_simulate3d(dummy, dummy, 4, 4, 4, dummy, 2, 2, 2, ctypes.byref(cfg), dummy, dummy, None, None, dummy,
                          need - 1, None)
    assert st == 6
    assert L.mpr_reference_curve3d(0.5, dummy, 4, 7, 10, 10, 0, dummy, dummy, 1 << 40, None) == 2   # odd L
    assert L.mpr_calibrate_temperature3d(dummy, dummy, 4, 4, 4, 2, 2, 2, 0.5, 1.0, dummy, dummy, 0, dummy, None,
                                         None, dummy, 1 << 40, None) == 1                          # no curve points


def test_per_chain_stop_workspace_holds_the_history():
    L = _lib.lib()
    a = _lib.SimConfig(n_real=256, stop_mode=_lib.STOP_AUTO, n_max=1000).to_c()
    b = _lib.SimConfig(n_real=256, stop_mode=_lib.STOP_AUTO_CHAIN, n_max=1000).to_c()
    wa = L.mpr_simulate_workspace_bytes(512, 512, 32, 32, ctypes.byref(a))
    wb = L.mpr_simulate_workspace_bytes(512, 512, 32, 32, ctypes.byref(b))
    assert wb - wa >= 1001 * 256 * 8
