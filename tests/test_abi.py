"""The C-ABI library loads, exports every symbol include/oim.h declares, and
rejects bad arguments on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "oim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(oim_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def oim():
    import paper_2505_22631_amd as m
    m.lib()
    return m


def test_every_declared_symbol_is_exported(oim):
    from paper_2505_22631_amd import _lib
    syms = _header_symbols()
    assert len(syms) >= 12
    L = _lib.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(_lib.PROTOTYPES), "binding prototypes and header disagree"


def _header_structs():
    """{typedef name: [field names in order]} of the header's structs."""
    text = open(os.path.join(ROOT, "include", "oim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            m = re.search(r"(\w+)\s*(\[[^\]]*\])?\s*$", decl.strip())
            if m and decl.strip():
                fields.append(m.group(1))
        out[name] = fields
    return out


def test_binding_structs_match_the_header(oim):
    # every struct the binding passes through the C ABI has the header's
    # fields in the header's order
    from paper_2505_22631_amd import _lib
    structs = _header_structs()
    pairs = {"oim_run_cfg": _lib.RunCfg, "oim_readout": _lib.Readout,
             "oim_adjoint_cfg": _lib.AdjointCfg, "oim_tune_report": _lib.TuneReport,
             "oim_problem_info": _lib.ProblemInfo}
    for cname, cls in pairs.items():
        assert cname in structs, cname
        assert [f for f, _ in cls._fields_] == structs[cname], cname


def test_abi_version_and_status_names(oim):
    from paper_2505_22631_amd import _lib
    assert oim.oim_abi_version() == _lib.ABI_VERSION == 4
    assert _lib.status_name(0) == "OIM_OK"
    assert _lib.status_name(3) == "OIM_E_ASYM"
    assert _lib.status_name(99) == "OIM_E_UNKNOWN"


def _csr_call(oim, n, rp, ci, J):
    L = oim.lib()
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, np.int64)
    ci = np.ascontiguousarray(ci, np.int32)
    J = np.ascontiguousarray(J, np.float32)
    st = L.oim_problem_from_csr(n, ci.size, rp.ctypes.data_as(ctypes.c_void_p),
                                ci.ctypes.data_as(ctypes.c_void_p),
                                J.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(h))
    return st, L.oim_last_error().decode()


def test_csr_validation_errors(oim):
    g = synth.erdos_renyi(30, 0.3, seed=1)
    rp, ci, J = g.row_ptr.copy(), g.col.copy(), (-g.w).copy()
    # bad sizes
    assert _csr_call(oim, 0, [0], [], [])[0] == 1
    # row_ptr[0] != 0
    bad = rp.copy(); bad[0] = 1
    assert _csr_call(oim, 30, bad, ci, J)[0] == 2
    # unsorted row
    c2 = ci.copy(); s, e = rp[0], rp[1]; c2[s:e] = c2[s:e][::-1]
    assert _csr_call(oim, 30, rp, c2, J)[0] == 2
    # out of range column
    c3 = ci.copy(); c3[-1] = 30
    assert _csr_call(oim, 30, rp, c3, J)[0] == 2
    # self loop
    tiny_rp, tiny_ci = [0, 1, 2], [0, 0]
    assert _csr_call(oim, 2, tiny_rp, tiny_ci, [1.0, 1.0])[0] == 2
    # asymmetric value
    J2 = J.copy(); J2[0] = 5.0
    st, msg = _csr_call(oim, 30, rp, ci, J2)
    assert st == 3 and "!=" in msg
    # missing transpose
    assert _csr_call(oim, 3, [0, 1, 1, 1], [1], [1.0])[0] == 3
    # non-finite
    J3 = J.copy(); J3[0] = np.nan
    assert _csr_call(oim, 30, rp, ci, J3)[0] == 4


def test_dense_validation_errors(oim):
    L = oim.lib()
    h = ctypes.c_void_p()
    A = np.zeros((4, 4), np.float32)
    A[0, 1] = 1.0
    st = L.oim_problem_from_dense(4, A.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(h))
    assert st == 3
    A[1, 0] = 1.0
    A[2, 3] = A[3, 2] = np.inf
    st = L.oim_problem_from_dense(4, A.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(h))
    assert st == 4
    st = L.oim_problem_from_dense(0, A.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(h))
    assert st == 1


def test_invalid_handles_and_args(oim):
    from paper_2505_22631_amd import _lib
    L = oim.lib()
    cfg = _lib.RunCfg(2, 1, 1, 0.01, 0, 0)
    assert L.oim_run(None, ctypes.byref(cfg), None, None, None, None, 0, None, None, None,
                     None) == 8
    assert L.oim_phase_from_theta(-1, None, None, None) == 1
    assert L.oim_theta_from_phase(3, None, None, None) == 1
    assert L.oim_round(1, 10, None, None, None) == 1
    assert L.oim_round(2, -1, None, None, None) == 1
    assert L.oim_round(2, 0, None, None, None) == 0
    assert L.oim_cut(None, 1, None, None, None, None) == 8
    assert L.oim_conflicts(None, 1, None, None, None) == 8
    assert L.oim_energy(None, 2, 1, None, None, None, None, None) == 8
    info = _lib.ProblemInfo()
    assert L.oim_problem_info_get(None, ctypes.byref(info)) == 8
    L.oim_problem_destroy(None)  # no-op


def test_valid_problem_without_gpu_reports_hip_error(oim):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g = synth.cycle(8)
    st, msg = _csr_call(oim, 8, g.row_ptr, g.col, -g.w)
    assert st == 7 and msg


def test_block_batch_validation(oim):
    L = oim.lib()
    a = synth.cycle(6)
    b = synth.cycle(4)
    # a proper block-diagonal batch passes validation (then fails on the missing GPU)
    rows = np.concatenate([a.row_ptr, a.row_ptr[-1] + b.row_ptr[1:]])
    cols = np.concatenate([a.col, b.col + 6]).astype(np.int32)
    J = -np.ones(cols.size, np.float32)
    off = np.array([0, 6, 10], np.int32)

    def call(offs, c=cols):
        h = ctypes.c_void_p()
        o = np.ascontiguousarray(offs, np.int32)
        c = np.ascontiguousarray(c, np.int32)
        rp = np.ascontiguousarray(rows, np.int64)
        return L.oim_problem_from_csr_blocks(10, c.size, rp.ctypes.data_as(ctypes.c_void_p),
                                             c.ctypes.data_as(ctypes.c_void_p),
                                             J.ctypes.data_as(ctypes.c_void_p), len(o) - 1,
                                             o.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(h))
    import torch
    if not torch.cuda.is_available():
        assert call(off) == 7
    assert call([0, 5, 10]) == 2           # an edge crosses the boundary
    assert call([0, 6, 6, 10]) == 1        # empty instance
    assert call([1, 6, 10]) == 1           # does not start at 0


def test_adjoint_entry_points_reject_bad_handles(oim):
    # host-side checks run before any device call
    from paper_2505_22631_amd import _lib
    L = oim.lib()
    cfg = _lib.AdjointCfg(2, 1, 10, 0.01, 4, 0)
    words = ctypes.c_int64(-1)
    assert L.oim_adjoint_checkpoint_words(None, ctypes.byref(cfg), ctypes.byref(words)) == 8
    assert L.oim_adjoint_forward(None, ctypes.byref(cfg), None, None, None, None, 0, None, None,
                                 None, None, None) == 8
    assert L.oim_adjoint_backward(None, ctypes.byref(cfg), None, None, None, None, 0, None, None,
                                  None, None, None) == 8
    assert "destroyed" in L.oim_last_error().decode()


def test_tuning_entry_points_reject_bad_handles(oim):
    from paper_2505_22631_amd import _lib
    L = oim.lib()
    cfg = _lib.RunCfg(2, 1, 10, 0.01, 0, 0)
    rep = _lib.TuneReport()
    assert L.oim_autotune(None, ctypes.byref(cfg), None, None, None, None, None, 5,
                          ctypes.byref(rep), None) == 8
    assert L.oim_set_tuning(None, 2, 64, 1, 4) == 8
