"""Host-side checks of the C ABI (no GPU): the library loads and exports every
function that include/zkvc.h declares, and the binding's structs match the
header's sizes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zkvc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(zkvc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def zk():
    from paper_2504_12217_amd import zkvc
    if not os.path.exists(zkvc.LIB_PATH):
        pytest.skip("library not built")
    return zkvc


def test_library_exports_every_declared_function(zk):
    lib = zk.lib()
    declared = _declared_functions()
    assert len(declared) >= 15
    missing = [f for f in declared if not hasattr(lib, f)]
    assert not missing, missing
    assert set(zk.EXPORTS) <= set(declared)


def test_struct_layouts_match_header(zk):
    assert ctypes.sizeof(zk.Fr) == 32
    assert ctypes.sizeof(zk.G1) == 64
    assert ctypes.sizeof(zk.G2) == 128
    assert ctypes.sizeof(zk.Proof) == 256
    assert ctypes.sizeof(zk.Shape) == 16
    assert ctypes.sizeof(zk.ProveJob) == 104  # 3 pointers, 2 zkvc_fr, 2 pointers
    assert ctypes.sizeof(zk.ServerConfig) == 16
    assert ctypes.sizeof(zk.ServerResult) == 24
    assert ctypes.sizeof(zk.ValuPeak) == 48  # 5 doubles, 1 uint32, padding
    text = open(HEADER).read()
    for name in ("ZKVC_PLAIN = 0", "ZKVC_CRPC_PSQ = 1", "ZKVC_PLAIN_ADD = 2", "ZKVC_PLAIN_PSQ = 3", "ZKVC_CRPC = 4"):
        assert name in text


def test_marshalling_round_trip(zk):
    v = (1 << 253) + 12345
    assert zk.words_to_int(zk.fr(v).l) == v
    p = zk.Proof()
    assert zk.proof_to_tuple(p) == (None, None, None)
    assert zk.proof_from_bytes(bytes(256)).A.x[0] == 0
    assert zk.vk_header(b"ZKVC-VK1" + bytes([1, 0, 0, 0, 4, 0, 0, 0, 8, 0, 0, 0, 4, 0, 0, 0, 0, 0, 0, 0, 8, 0, 0, 0])) \
        == (4, 8, 4, 0, 8)


def test_prove_batch_rejects_empty_batch_before_device_work(zk):
    assert zk.lib().zkvc_prove_batch(None, 0, None) == zk.EINVAL


def test_server_argument_errors_before_device_work(zk):
    lib = zk.lib()
    assert lib.zkvc_server_create(None, None) == zk.EINVAL
    cfg = zk.ServerConfig(0, 0)
    h = ctypes.c_void_p()
    assert lib.zkvc_server_create(ctypes.byref(cfg), ctypes.byref(h)) == zk.EINVAL
    assert lib.zkvc_server_submit(None, None, None) == zk.EINVAL
    assert lib.zkvc_server_wait(None, 1, None) == zk.EINVAL
    assert lib.zkvc_server_destroy(None) == zk.OK


def test_tuning_table_import_export_round_trip(zk):
    before = zk.tune_export()
    try:
        zk.tune_import("msm_g1 16 11\nmsm_kdiv 20 15\nntt 16 8\n")
        got = set(zk.tune_export().splitlines())
        assert {"msm_g1 16 11", "msm_kdiv 20 15", "ntt 16 8"} <= got
        for bad in ("msm_g1 16 40", "ntt 30 8", "bogus 1 2", "msm_g1 16"):
            with pytest.raises(zk.ZkvcError) as e:
                zk.tune_import(bad)
            assert e.value.code == zk.EINVAL
        # a rejected text changes nothing
        assert {"msm_g1 16 11", "msm_kdiv 20 15", "ntt 16 8"} <= set(zk.tune_export().splitlines())
    finally:
        zk.tune_import("msm_g1 16 0\nmsm_kdiv 20 0\nntt 16 0\n")
        zk.tune_import(before)
    assert zk.lib().zkvc_autotune(8, 10, 12, None) == zk.EINVAL  # unknown target, before device work
    assert zk.lib().zkvc_autotune(1, 12, 10, None) == zk.EINVAL


def test_strerror_without_gpu(zk):
    # strerror only formats text; no device work
    assert zk.lib().zkvc_strerror(zk.EINVAL)


def test_graph_switch_and_profile_selection_are_host_only(zk):
    """zkvc_set_graphs returns the previous setting; zkvc_profile_select checks its list length."""
    prev = zk.set_graphs(1)
    try:
        assert zk.set_graphs(0) == 1
        assert zk.set_graphs(0) == 0
    finally:
        zk.set_graphs(prev)
    zk.profile_select(["msm_acc_points_g1", "ntt_pass"])
    zk.profile_select("ntt_pass")
    zk.profile_select(None)
    with pytest.raises(zk.ZkvcError) as e:
        zk.profile_select("k" * 5000)
    assert e.value.code == zk.EINVAL
