"""The C-ABI library without a GPU: it loads, exports every entry point the
header declares, and its host-only logic (config defaults, Table 2 features,
argument checks) behaves; device calls on a GPU-less host fail cleanly."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _mlmq():
    import paper_2602_10080_amd as mlmq
    return mlmq


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mlmq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlmq_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    mlmq = _mlmq()
    lib = mlmq.lib()
    names = declared_symbols()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(mlmq.EXPORTS)


def test_struct_sizes_match_header(tmp_path):
    """The binding's structures have the sizes a C compiler gives the
    header's (the library rejects a config whose struct_size differs)."""
    mlmq = _mlmq()
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "mlmq.h"\nint main(void) { printf("%zu %zu %zu", '
                   'sizeof(mlmq_config), sizeof(mlmq_stats), sizeof(mlmq_features)); return 0; }\n')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    sizes = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert sizes == [ctypes.sizeof(mlmq.Config), ctypes.sizeof(mlmq.Stats), ctypes.sizeof(mlmq.Features)]


def test_config_default_and_struct_size_check():
    mlmq = _mlmq()
    c = mlmq.default_config()
    d = c.as_dict()
    assert d["wg_size"] == 64 and d["l1_type"] == mlmq.L1_VEC and d["l2_type"] == mlmq.L2_FIFO
    bad = mlmq.Config()
    bad.struct_size = 12
    assert mlmq.lib().mlmq_config_default(ctypes.byref(bad)) == mlmq.ERR_INVALID_ARG
    assert b"struct_size" in mlmq.lib().mlmq_last_error()


@pytest.mark.parametrize("kind", ["grid", "rmat", "uniform"])
def test_features_match_numpy(kind):
    mlmq = _mlmq()
    g = {"grid": lambda: gg.grid(50, 70, 0.1, seed=2), "rmat": lambda: gg.rmat(11, 8, seed=3),
         "uniform": lambda: gg.uniform(3000, 20000, seed=4)}[kind]()
    f = mlmq.features(g)
    deg = g.degrees().astype(np.float64)
    w = g.w.astype(np.float64)
    want = dict(n=g.n, nnz=g.m, avg_deg=deg.mean(), max_deg=deg.max(), std_deg=deg.std(),
                avg_w=w.mean(), std_w=w.std(), max_w=w.max())
    for k, v in want.items():
        assert f[k] == pytest.approx(v, rel=1e-9, abs=1e-9), k


def test_features_reject_bad_csr():
    mlmq = _mlmq()
    off = np.array([0, 2, 1, 3], np.int32)
    col = np.array([0, 1, 2], np.int32)
    w = np.ones(3, np.uint32)
    f = mlmq.Features()
    rc = mlmq.lib().mlmq_features_host(3, 3, off.ctypes.data, col.ctypes.data, w.ctypes.data, ctypes.byref(f))
    assert rc == mlmq.ERR_INVALID_ARG
    off = np.array([0, 1, 2, 3], np.int32)
    col = np.array([0, 1, 3], np.int32)
    rc = mlmq.lib().mlmq_features_host(3, 3, off.ctypes.data, col.ctypes.data, w.ctypes.data, ctypes.byref(f))
    assert rc == mlmq.ERR_INVALID_ARG


def test_device_calls_fail_cleanly_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    mlmq = _mlmq()
    g = gg.grid(4, 4)
    h = ctypes.c_void_p()
    off = g.off32()
    rc = mlmq.lib().mlmq_graph_create(g.n, g.m, off.ctypes.data, g.col.ctypes.data, g.w.ctypes.data, 0,
                                      ctypes.byref(h))
    assert rc == mlmq.ERR_DEVICE and not h
    # flags are checked before the device: unknown bits, or keep-order with degree-order
    for flags in (8, mlmq.GRAPH_KEEP_ORDER | mlmq.GRAPH_DEGREE_ORDER):
        rc = mlmq.lib().mlmq_graph_create(g.n, g.m, off.ctypes.data, g.col.ctypes.data, g.w.ctypes.data, flags,
                                          ctypes.byref(h))
        assert rc == mlmq.ERR_INVALID_ARG and not h
    assert mlmq.lib().mlmq_sssp(None, 0, None, None) == mlmq.ERR_INVALID_ARG
    assert mlmq.lib().mlmq_check(None, 0, None, None, None, None) == mlmq.ERR_INVALID_ARG
