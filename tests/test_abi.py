"""The C ABI library builds, loads without a GPU and exports every function
that include/sdsl.h declares (no compute calls here)."""
import ctypes as C
import os
import re

import paper_2604_23979_amd as sd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "sdsl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdsl_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for must in ("sdsl_setup", "sdsl_refactor", "sdsl_update_values", "sdsl_solve", "sdsl_solve_batch",
                 "sdsl_destroy", "sdsl_get_info", "sdsl_last_error", "sdsl_default_options"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = C.CDLL(sd.LIB_PATH)
    for name in header_functions():
        assert hasattr(L, name), name
    assert set(header_functions()) == set(sd.SIGNATURES)


def test_default_options_and_footprint_host_only():
    o = sd._binding.COptions()
    sd.lib().sdsl_default_options(C.byref(o))
    assert o.method == sd.BJ and o.pivot == sd.PIVOT_SHIFT and o.max_iter == 100000 and o.check_every == 16
    assert abs(o.inner_tol - 1e-4) < 1e-18
    import numpy as np
    rp = np.array([0, 1, 2], dtype=np.int64)
    A = sd._binding.CSR(2, 2, rp.ctypes.data_as(C.c_void_p), None, None, sd._binding.MEM_HOST)
    bp = np.array([0, 2], dtype=np.int32)
    part = sd._binding.Partition(1, bp.ctypes.data_as(C.c_void_p), 0)
    assert sd.lib().sdsl_footprint_bytes(C.byref(A), C.byref(part), C.byref(o), None) > 0


def test_footprint_counts_gmres_basis_and_bbd_tail_factors_host_only():
    """The admission prediction grows by at least the GMRES basis for GMRES
    and by the dense Schur complement and its inverse plus the tail factors
    (per block: tail rows x (distinct border columns + rows)) for BBD.  The
    tails come from the oracle, the distinct counts from the pattern.  A BBD
    prediction needs the pattern on the host: without it, or for a pattern
    that is not bordered block diagonal, the answer is 0."""
    import numpy as np

    import oracle as O
    from ipm_inputs import gen
    from paper_2604_23979_amd.serve import footprint

    s = gen.bbd_system(nblocks=3, block_rows=60, n_border=12, nnz_off=4, half_band=10, tail_frac=0.2,
                       border_c=2, seed=14, name="bbd-tiny")
    n, nbd = s.n, s.n_border
    ni = n - nbd
    pcg = footprint(s, sd.Options(spd=False))
    gm = footprint(s, sd.Options(krylov=sd.GMRES, spd=False, restart=30))
    bbd = footprint(s, sd.Options(method=sd.BBD, krylov=sd.GMRES, spd=False, restart=30))
    assert gm >= pcg + (2 * 30 + 1) * n * 8
    tails = O.BBD(s).parts()["tail"]
    M = s.scipy().tocsr()
    hg = 0
    for b in range(s.nblocks):
        lo, hi = int(s.block_ptr[b]), int(s.block_ptr[b + 1])
        ne = np.unique(M[lo:hi, ni:].nonzero()[1]).size
        nf = np.unique(M[ni:, lo:hi].nonzero()[0]).size
        hg += (hi - int(tails[b])) * (ne + nf)
    assert bbd >= gm + 2 * nbd * nbd * 8 + 8 * hg
    o = sd.Options(method=sd.BBD, krylov=sd.GMRES, spd=False).c()
    rp = np.ascontiguousarray(s.row_ptr, dtype=np.int64)
    bp = np.ascontiguousarray(s.block_ptr, dtype=np.int32)
    part = sd._binding.Partition(s.nblocks, bp.ctypes.data_as(C.c_void_p), nbd)
    A = sd._binding.CSR(n, s.nnz, rp.ctypes.data_as(C.c_void_p), None, None, sd._binding.MEM_HOST)
    assert sd.lib().sdsl_footprint_bytes(C.byref(A), C.byref(part), C.byref(o), None) == 0
    bad = M.tolil()
    bad[0, 70] = 1.0  # block 0 row -> block 1 column
    bad = bad.tocsr()
    bad.sort_indices()
    s_bad = gen.System("bad", bad.indptr.astype(np.int64), bad.indices.astype(np.int32), bad.data, s.b,
                       s.block_ptr, n_border=nbd)
    assert footprint(s_bad, sd.Options(method=sd.BBD, krylov=sd.GMRES, spd=False)) == 0


def test_setup_rejects_bad_arguments_without_touching_the_device():
    o = sd._binding.COptions()
    sd.lib().sdsl_default_options(C.byref(o))
    h = C.c_void_p()
    assert sd.lib().sdsl_setup(None, None, C.byref(o), None, None, None, C.byref(h)) == sd.E_INVALID
    assert b"null" in sd.lib().sdsl_last_error(None)
    assert not h.value
    # an allocator needs both functions (checked before any device work)
    import numpy as np
    rp = np.array([0, 1, 2], dtype=np.int64)
    ci = np.array([0, 1], dtype=np.int32)
    v = np.array([1.0, 1.0])
    A = sd._binding.CSR(2, 2, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
                        v.ctypes.data_as(C.c_void_p), sd._binding.MEM_HOST)
    bp = np.array([0, 2], dtype=np.int32)
    part = sd._binding.Partition(1, bp.ctypes.data_as(C.c_void_p), 0)
    half = sd._binding.Allocator(sd._binding.ALLOC_FN(lambda nbytes, s, ctx: None), sd._binding.FREE_FN(), None)
    assert sd.lib().sdsl_setup(C.byref(A), C.byref(part), C.byref(o), None, C.byref(half), None,
                               C.byref(h)) == sd.E_INVALID
    assert b"allocator" in sd.lib().sdsl_last_error(None)
    assert not h.value


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; --gpus N > 1 exits with a message
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
