"""The block product on library-held scratch (smfs_apply_block_noalloc)
against the block product on a caller workspace (smfs_apply_block), through
the C-ABI: two calls in a row, the second on a smaller problem with fewer
right-hand sides (the scratch keeps the first call's contents)."""
import ctypes as C

import numpy as np
import pytest

from oracle import geometry as geo, mfs
from paper_2407_03343_amd import workloads as wl

from gpu_common import _say, _import_oracle_factors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SMALL = dict(n_proxy=60, n_colloc_base=80, n_image=4, n_check_base=0)


def _noalloc(dev):
    L = dev.lib()
    f = L.smfs_apply_block_noalloc
    f.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    f.restype = C.c_int
    g = L.smfs_noalloc_scratch_bytes
    g.argtypes = []
    g.restype = C.c_size_t
    return f, int(g())


def _problem(dev, c):
    g = geo.build(c, 1.0, geo.Params(**SMALL))
    pbo = mfs.Problem(g).setup()
    lib = dev.Problem(c, 1.0, **SMALL).bind()
    _import_oracle_factors(lib, pbo)
    return lib


def _centres12():
    rng = np.random.default_rng(41)
    c = [np.array([0.0, 0.0, 0.0]), np.array([2.002, 0.0, 0.0]),
         np.array([0.0, 4.0, 0.0]), np.array([0.0, 6.05, 0.0])]
    while len(c) < 12:
        x = rng.uniform(-6, 8, 3)
        if all(np.linalg.norm(x - y) > 2.4 for y in c):
            c.append(x)
    return np.array(c)


def test_noalloc_block_product_matches_workspace_form(dev):
    fn, cap = _noalloc(dev)
    _say(f"no-alloc block product: scratch {cap} bytes")
    cases = [(_centres12(), 9), (np.array([[0.0, 0, 0], [2.05, 0.3, 0.0], [0.4, 2.3, 0.1]]), 2)]
    for call, (c, nrhs) in enumerate(cases):
        lib = _problem(dev, c)
        n = 3 * lib.T
        _say(f"  call {call}: {len(c)} spheres, T={lib.T}, nrhs={nrhs}, "
             f"workspace form needs {lib.block_workspace_bytes(nrhs)} bytes")
        assert lib.block_workspace_bytes(nrhs) <= cap
        M = torch.from_numpy(np.stack([wl.random_vector(n, 90 + q) for q in range(nrhs)])).cuda()
        ref = lib.apply_block(M)
        Y = torch.full_like(M, np.nan)
        rc = fn(lib.h, nrhs, C.c_void_p(M.data_ptr()), C.c_void_p(Y.data_ptr()), n,
                C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0, dev.lib().smfs_last_error().decode()
        torch.cuda.synchronize()
        a, b = Y.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a, b), np.abs(a - b).max()


def test_noalloc_rejects_too_large(dev):
    fn, cap = _noalloc(dev)
    lib = _problem(dev, _centres12())
    n = 3 * lib.T
    nrhs = 1
    while lib.block_workspace_bytes(nrhs) <= cap:
        nrhs *= 2
    _say(f"no-alloc block product: nrhs {nrhs} needs {lib.block_workspace_bytes(nrhs)} > {cap} bytes")
    M = torch.zeros(nrhs, n, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(M)
    rc = fn(lib.h, nrhs, C.c_void_p(M.data_ptr()), C.c_void_p(Y.data_ptr()), n,
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -4                       # SMFS_E_NOMEM, nothing launched
    assert "scratch" in dev.lib().smfs_last_error().decode()
