"""Driver of the host sanitizer test (run in a subprocess with the
AddressSanitizer runtime preloaded): exercises the host-side grid builder and
C-ABI glue of libsgcm (a host-only sanitizer build of grid.cpp and capi.cpp)
and the oracle (a sanitizer build of its source) on small cases, including
invalid arguments.  Prints "asan ok" when every call returned."""
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402  (loads SGCM_ORACLE_LIB)
from paper_1507_04769_amd import workloads as W  # noqa: E402


def grid_glue(path):
    L = ctypes.CDLL(path)
    L.sgcm_grid_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_void_p)]
    L.sgcm_grid_size.restype = ctypes.c_int64
    L.sgcm_grid_size.argtypes = [ctypes.c_void_p]
    L.sgcm_grid_nodes.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.sgcm_grid_keys.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.sgcm_grid_destroy.argtypes = [ctypes.c_void_p]
    L.sgcm_strerror.restype = ctypes.c_char_p
    for d, level in ((1, 0), (1, 5), (2, 5), (3, 4), (6, 0), (6, 1), (6, 4), (6, 5), (8, 3)):
        lo = np.full(d, -1.0)
        hi = np.full(d, 2.0)
        g = ctypes.c_void_p()
        assert L.sgcm_grid_create(d, level, lo.ctypes.data, hi.ctypes.data, ctypes.byref(g)) == 0
        M = L.sgcm_grid_size(g)
        nodes = np.empty((M, d))
        keys = np.empty((M, d), dtype=np.int32)
        assert L.sgcm_grid_nodes(g, nodes.ctypes.data) == 0
        assert L.sgcm_grid_keys(g, keys.ctypes.data) == 0
        assert np.all(nodes >= -1.0 - 1e-12) and np.all(nodes <= 2.0 + 1e-12)
        L.sgcm_grid_destroy(g)
    g = ctypes.c_void_p()
    lo = np.zeros(6)
    assert L.sgcm_grid_create(0, 2, lo.ctypes.data, lo.ctypes.data, ctypes.byref(g)) != 0
    assert L.sgcm_grid_create(6, -1, lo.ctypes.data, lo.ctypes.data, ctypes.byref(g)) != 0
    assert L.sgcm_grid_create(6, 2, lo.ctypes.data, lo.ctypes.data, None) != 0
    assert L.sgcm_grid_create(2, 6, lo.ctypes.data, lo.ctypes.data, ctypes.byref(g)) != 0  # above the finest level
    assert L.sgcm_grid_create(9, 1, lo.ctypes.data, lo.ctypes.data, ctypes.byref(g)) != 0  # above the largest d
    assert L.sgcm_grid_nodes(None, None) != 0 and L.sgcm_grid_size(None) == -1
    L.sgcm_grid_destroy(None)
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert L.sgcm_strerror(code)


def oracle_paths():
    gr = O.grid(6, 3, W.BOX_LO, W.BOX_HI)
    vals = W.random_values(len(gr.nodes), 3, seed=5)
    w = O.build_surplus(6, 3, vals)
    xq = W.uniform_in_box(40, seed=6)
    a = O.eval_hier(6, 3, w, xq, W.BOX_LO, W.BOX_HI)
    assert np.all(np.isfinite(a))
    x0 = W.uniform_in_box(4, seed=7)
    x0[1, 2] = np.nan
    for kw in (dict(N=7, T=2.0), dict(N=1, T=0.5, max_iter=0), dict(N=5, T=2.0, scheme=O.LOBATTO4),
               dict(m=2, B=W.input_matrix(2), N=6, T=5.0, max_iter=30, continuation=2)):
        r = O.solve_bvps(O.Problem(**kw), x0, want_traj=True)
        assert r.status[1] == O.NONFINITE
    c = np.random.default_rng(8).standard_normal((9, 3))
    O.total_error(c, c + 1e-3, c + 2e-3, order=6)
    O.total_error(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)))


if __name__ == "__main__":
    grid_glue(sys.argv[1])
    oracle_paths()
    print("asan ok", flush=True)
