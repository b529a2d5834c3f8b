"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/lnv.h, and rejects bad arguments on the host before any
launch (status codes of include/lnv.h)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lnv.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lnv_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2002_07704_amd import lib as L
    return L.load()


def test_exports_every_declared_symbol(lib):
    from paper_2002_07704_amd import lib as L
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, n


def test_strerror_codes(lib):
    assert lib.lnv_strerror(0) == b"success"
    assert b"capacity" in lib.lnv_strerror(2)
    assert lib.lnv_strerror(99) == b"unknown status"


def test_host_side_argument_errors(lib):
    from paper_2002_07704_amd import lib as L
    box = (ctypes.c_double * 3)(10.0, 10.0, 10.0)
    nnz = ctypes.c_int64(0)
    # null positions / non-positive atom count / negative range
    assert lib.lnv_neighbours(None, 4, box, 3.0, ctypes.c_void_p(8), None, 0, ctypes.byref(nnz), None) == L.EINVAL
    assert lib.lnv_neighbours(ctypes.c_void_p(8), 0, box, 3.0, ctypes.c_void_p(8), None, 0, ctypes.byref(nnz), None) == L.EINVAL
    assert lib.lnv_neighbours(ctypes.c_void_p(8), 4, box, -1.0, ctypes.c_void_p(8), None, 0, ctypes.byref(nnz), None) == L.EINVAL
    bad = (ctypes.c_double * 3)(10.0, 0.0, 10.0)
    assert lib.lnv_neighbours(ctypes.c_void_p(8), 4, bad, 3.0, ctypes.c_void_p(8), None, 0, ctypes.byref(nnz), None) == L.EINVAL
    # multiply with missing matrices / unsupported block edge / missing tables
    assert lib.lnv_bsm_multiply(1.0, None, None, 0, 0.0, None, None) == L.EINVAL
    p = L.LnvPattern(n=4, n_items=1, nnzb=4, row_ptr=8, col=8, items=8)
    m = L.LnvBsm(pat=ctypes.pointer(p), blk=4, dtype=L.F64, val=8)
    m5 = L.LnvBsm(pat=ctypes.pointer(p), blk=5, dtype=L.F64, val=8)
    assert lib.lnv_bsm_multiply(1.0, ctypes.byref(m5), ctypes.byref(m), 0, 0.0, ctypes.byref(m), None) == L.EUNSUPPORTED
    assert lib.lnv_bsm_multiply(1.0, ctypes.byref(m), ctypes.byref(m), 0, 0.0, ctypes.byref(m), None) == L.EPATTERN
    q = L.LnvPattern(n=5, n_items=1, nnzb=4, row_ptr=8, col=8, items=8)
    q.ix.tab = 8
    mq = L.LnvBsm(pat=ctypes.pointer(q), blk=4, dtype=L.F64, val=8)
    assert lib.lnv_bsm_multiply(1.0, ctypes.byref(m), ctypes.byref(mq), 0, 0.0, ctypes.byref(m), None) == L.EPATTERN
    # op(B): 0, 1, or 2 (B symmetric, its half stored: atom tiles only, no traces)
    pb = L.LnvPattern(n=4, n_items=1, nnzb=4, row_ptr=8, col=8, items=8)
    pb.ix.tab = 8
    mb = L.LnvBsm(pat=ctypes.pointer(pb), blk=4, dtype=L.F64, val=8)
    for tb in (-1, 3):
        assert lib.lnv_bsm_multiply(1.0, ctypes.byref(m), ctypes.byref(mb), tb, 0.0, ctypes.byref(m), None) == L.EINVAL
    assert lib.lnv_bsm_multiply(1.0, ctypes.byref(m), ctypes.byref(mb), 2, 0.0, ctypes.byref(m), None) == L.EUNSUPPORTED
    # CG step: bad options are rejected before anything else
    o = L.LnvOpts(0, 1e-11, 0.1)
    assert lib.lnv_cg_step(None, None, None, None, 8.0, 0, ctypes.byref(o), None, None) == L.EINVAL
    o = L.LnvOpts(40, 1e-11, 0.1)
    assert lib.lnv_cg_step(ctypes.byref(m), ctypes.byref(m), ctypes.byref(m), None, 8.0, 0, ctypes.byref(o), None, None) == L.EINVAL
    assert lib.lnv_hotelling(ctypes.byref(m), ctypes.byref(m), -1, None, None) == L.EINVAL
    assert lib.lnv_adjoint(None, None, None, None, None, None, None, None) == L.EINVAL
    ws = L.LnvAdjWs()
    assert lib.lnv_adjoint(ctypes.byref(m), ctypes.byref(m), ctypes.byref(m), None, None, None,
                           ctypes.byref(ws), None) == L.EINVAL
    box = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    assert lib.lnv_forces(None, box, None, None, None, 1, 1.0, None, None, 0.0, 12.0, 3.0, None,
                          14.0, 2.5, 1, None, None, None, None, None) == L.EINVAL
    assert lib.lnv_partials_len(10) >= 12 * 8 * 1024
    # occupation bounds: missing work/out, steps outside [1, 64], block edge
    work = ctypes.c_void_p(8)
    assert lib.lnv_occupation_bounds(ctypes.byref(m), ctypes.byref(m), 16, None, work, None) == L.EINVAL
    assert lib.lnv_occupation_bounds(ctypes.byref(m), ctypes.byref(m), 0, work, work, None) == L.EINVAL
    assert lib.lnv_occupation_bounds(ctypes.byref(m), ctypes.byref(m), 65, work, work, None) == L.EINVAL
    assert lib.lnv_occupation_bounds(ctypes.byref(m5), ctypes.byref(m), 16, work, work, None) == L.EUNSUPPORTED
    assert lib.lnv_occupation_bounds(ctypes.byref(m), ctypes.byref(mq), 16, work, work, None) == L.EPATTERN
    assert lib.lnv_lanczos_len(0) == 0 and lib.lnv_lanczos_len(10) >= 5 * 40 + 128
    assert lib.lnv_cg_check(None, None, None) == L.EINVAL


def test_struct_layouts_match_header(tmp_path):
    """sizeof of every ABI struct, compiled from include/lnv.h by gcc, equals
    the ctypes mirror used by the binding."""
    import shutil
    import subprocess
    from paper_2002_07704_amd import lib as L
    if shutil.which("gcc") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("gcc or ROCm headers not available")
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "lnv.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %zu %zu", sizeof(lnv_pattern), sizeof(lnv_bsm),'
                   ' sizeof(lnv_eval_ws), sizeof(lnv_cg_ws), sizeof(lnv_opts),'
                   ' sizeof(lnv_adj_ws), sizeof(lnv_eval32_ws)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(x) for x in (L.LnvPattern, L.LnvBsm, L.LnvEvalWs, L.LnvCgWs, L.LnvOpts,
                                           L.LnvAdjWs, L.LnvEval32Ws)]
    assert got == want


def test_split_rows_cover_every_function_once():
    """Stored-row layout of atoms with 13/9/4 (and odd) function counts: each
    function of each atom lands in exactly one (row, slot), rows of an atom
    are consecutive, and only the last row of an atom is padded."""
    import numpy as np
    from paper_2002_07704_amd.system import split_rows
    nfun = np.array([13, 4, 9, 4, 1, 16, 5])
    atom_of, off_of = split_rows(nfun)
    seen = {}
    for i, (a, o) in enumerate(zip(atom_of, off_of)):
        for r in range(4):
            if o + r < nfun[a]:
                seen.setdefault((a, o + r), []).append((i, r))
    assert sorted(seen) == [(a, f) for a in range(len(nfun)) for f in range(nfun[a])]
    assert all(len(v) == 1 for v in seen.values())
    assert np.all(np.diff(atom_of) >= 0)
    assert list(np.bincount(atom_of)) == [4, 1, 3, 1, 1, 4, 2]
