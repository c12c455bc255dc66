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


def test_batched_workspace_covers_both_kernels():
    """Host-only size queries: a scene that the realization-lane sweep takes needs exactly its single-scene
    workspace inside a batch; with sweep_kernel = TILES (or few realizations) the batch needs the persistent tile
    batch's; a mixed batch needs the larger of the two."""
    L = _lib.lib()
    auto = _lib.SimConfig(n_real=64).to_c()
    tiles = _lib.SimConfig(n_real=64, sweep_kernel=_lib.SWEEP_TILES).to_c()
    few = _lib.SimConfig(n_real=8).to_c()
    big, small = (1024, 800), (70, 130)

    def batch(shapes):
        arr = (_lib.mpr_scene * len(shapes))()
        for i, (H, W) in enumerate(shapes):
            arr[i] = _lib.mpr_scene(H, W, 16, 16, i, None, None, None, None, None, None)
        return arr, len(shapes)

    single_lanes = L.mpr_simulate_workspace_bytes(*big, 16, 16, ctypes.byref(auto))
    single_tiles = L.mpr_simulate_workspace_bytes(*big, 16, 16, ctypes.byref(tiles))
    assert single_lanes != single_tiles                      # the lane sweep takes the large scene
    assert L.mpr_simulate_batched_workspace_bytes(*batch([big]), ctypes.byref(auto)) == single_lanes
    tile_only = L.mpr_simulate_batched_workspace_bytes(*batch([big]), ctypes.byref(tiles))
    assert tile_only > 0 and tile_only != single_lanes
    small_only = L.mpr_simulate_batched_workspace_bytes(*batch([small]), ctypes.byref(auto))
    assert small_only == L.mpr_simulate_batched_workspace_bytes(*batch([small]), ctypes.byref(tiles))
    assert (L.mpr_simulate_batched_workspace_bytes(*batch([big, small]), ctypes.byref(auto))
            == max(single_lanes, small_only))
    assert (L.mpr_simulate_batched_workspace_bytes(*batch([big, small]), ctypes.byref(few))
            == L.mpr_simulate_batched_workspace_bytes(*batch([big, small]),
                                                      ctypes.byref(_lib.SimConfig(n_real=8, sweep_kernel=_lib.SWEEP_TILES).to_c())))
