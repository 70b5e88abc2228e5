"""CPU-side checks of the C-ABI library: it loads, it exports every symbol
that include/qpx.h declares, and host-side argument validation rejects bad
calls before anything would reach a GPU."""
import ctypes
import os
import re

import pytest

import paper_2605_17913_amd as qpx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["qp_solve", "qp_backward", "qp_serve_submit", "qp_serve_poll"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = qpx.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(qpx.EXPORTS)


def test_default_opts():
    o = qpx.default_opts()
    assert o.form == 0 and o.max_iter == 100 and abs(o.tol - 1e-5) < 1e-12
    assert o.pc == 1 and abs(o.sigma - 0.1) < 1e-7 and abs(o.kappa_relax - 1e-4) < 1e-10
    assert o.assembly == qpx.ASSEMBLY["auto"]
    assert o.fp64_residual == qpx.RESIDUAL["auto"] and o.backoff == 0.0
    assert abs(o.relax_tol - 1e-6) < 1e-12 and o.relax_max_iter == 30


def test_status_strings_are_distinct():
    # return codes and per-QP status words have their own functions; no two
    # codes share a description
    L = qpx.lib()
    codes = [0, 1, -1, -2, -3, -4, -5]
    names = [L.qp_status_string(c) for c in codes]
    assert len(set(names)) == len(codes)
    assert L.qp_status_string(1) == b"pending"
    words = {}
    for outcome in range(4):
        for stage in range(8):
            words[(outcome, stage)] = L.qp_result_string(outcome | (stage << 8))
    assert len(set(words.values())) == len(words)
    assert words[(1, 0)] == b"iteration limit reached"
    assert words[(2, 2)] == b"non-finite value (stage: predictor)"
    # the precision bits do not change the description
    assert L.qp_result_string(0 | (1 << 16) | (1 << 17)) == words[(0, 0)]
    assert L.qp_result_string(7) == b"unknown per-QP status"
    assert qpx.result_string(3 | (6 << 8)).endswith("(stage: relax)")


def _struct_fields(name):
    import re
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{([^{}]*)\} " + name + ";", text).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            names += [re.findall(r"\w+", piece)[-1] for piece in decl.split(",")]
    return names


def test_binding_structs_match_the_header():
    # the ctypes mirrors must list the header's fields in the header's order
    for cname, py in (("qp_batch", qpx._Batch), ("qp_opts", qpx._Opts), ("qp_out", qpx._Out),
                      ("qp_grads", qpx._Grads), ("qp_server_opts", qpx._ServerOpts),
                      ("qp_timing", qpx._Timing), ("qp_plan", qpx._Plan)):
        assert _struct_fields(cname) == [f[0] for f in py._fields_], cname


def test_null_arguments_are_rejected_on_the_host():
    L = qpx.lib()
    o = qpx.default_opts()
    bt = qpx._Batch(4, 3, 2, 1, None, None, None, None, None, None)
    out = qpx._Out()
    # NULL context
    assert L.qp_solve(None, ctypes.byref(bt), ctypes.byref(o), ctypes.byref(out), None) == -1
    assert L.qp_backward(None, ctypes.byref(bt), ctypes.byref(o), ctypes.byref(out), None, None,
                         None, ctypes.byref(qpx._Grads()), None, None) == -1
    h = ctypes.c_void_p()
    assert L.qp_create(None, 0) == -1
    assert L.qp_status_string(-5) == b"unsupported size"
    assert L.qp_destroy(None) == 0


def test_cpu_tensors_raise():
    import torch
    Q = torch.eye(3).unsqueeze(0)
    with pytest.raises(qpx.QPError):
        qpx.solve(Q, torch.zeros(1, 3), None, None, None, None)


# static LDS of the kernels (context table; profiling counters), the bound the
# launch planning reserves next to each QP's dynamic LDS
STATIC_LDS = 512


def test_launch_plans():
    # host-side planning (no device call): border cap, threads per QP, factor
    # placement, assembly arithmetic and size limits
    c1 = qpx.plan(10, 20, 2)
    assert c1["threads"] == 128 and c1["kb"] == 10 and c1["factor_in_lds"]
    assert c1["assembly"] == "fp32" and c1["workspace_bytes"] == 0
    c2 = qpx.plan(50, 100, 10)
    assert c2["threads"] == 256 and c2["kb"] == 50 and c2["factor_in_lds"]
    assert 3 * (c2["lds_bytes"] + STATIC_LDS) <= 160 * 1024  # three QPs per CU
    c3 = qpx.plan(100, 200, 20)
    # the factor would fit LDS (131 KB) but leave one QP per CU; in global
    # memory four fit (register-limited: four waves per SIMD for systems of
    # 129 to 256 rows), with the same border
    assert c3["kb"] == 100 and not c3["factor_in_lds"] and c3["assembly"] == "mfma_fp32"
    assert c3["threads"] == 256 and (c3["lds_bytes"] + STATIC_LDS) * 4 <= 160 * 1024
    assert c3["workspace_bytes"] > 0
    # residency rule: the factor leaves LDS only when that at least doubles
    # the QPs per CU (capped at 12 waves per CU below 512 threads)
    small = qpx.plan(30, 60, 3)
    assert small["threads"] == 128 and small["factor_in_lds"]
    mid = qpx.plan(80, 160, 8)
    assert mid["threads"] == 256 and not mid["factor_in_lds"] and mid["kb"] == 80
    assert (mid["lds_bytes"] + STATIC_LDS) * 3 <= 160 * 1024
    narrow = qpx.plan(50, 100, 10, block=128)
    assert not narrow["factor_in_lds"] and narrow["kb"] == 50
    assert (narrow["lds_bytes"] + STATIC_LDS) * 6 <= 160 * 1024
    c5 = qpx.plan(256, 512, 32)
    # factor in global memory: every row with v > 0 may be bordered
    assert not c5["factor_in_lds"] and c5["kb"] == 512 and c5["threads"] == 512
    assert c5["assembly"] == "mfma_fp32" and c5["workspace_bytes"] > 1 << 20
    assert qpx.plan(256, 512, 32, kmax=256)["kb"] == 256
    # the standard form and the first partially condensed form border nothing
    assert qpx.plan(50, 100, 10, form="standard")["kb"] == 0
    assert qpx.plan(256, 512, 32, form="condensed")["kb"] == 0
    assert qpx.plan(256, 512, 32, form="standard")["assembly"] == "fp32"
    assert qpx.plan(128, 256, 16, assembly="bf16x3")["assembly"] == "bf16x3"
    # explicit block sizes: more than 512 rows need 512 threads
    with pytest.raises(qpx.QPError):
        qpx.plan(256, 512, 32, block=256)
    with pytest.raises(qpx.QPError):
        qpx.plan(1000, 10, 30)  # n + p beyond 1024 bordered rows
    with pytest.raises(qpx.QPError):
        qpx.plan(10, 5000, 1)   # m beyond 4096
    with pytest.raises(qpx.QPError):
        qpx.plan(10, 5, 10)     # p >= n


def test_planned_lds_fits_a_cu():
    # every plan's dynamic LDS plus the kernels' static LDS fits one CU's
    # 160 KiB, across shapes from tiny to the largest supported systems
    for n in (1, 7, 16, 50, 63, 64, 65, 100, 128, 200, 256, 400, 500):
        for mr in (0.5, 1, 2, 4):
            m = max(1, int(mr * n))
            for p in (0, n // 10, n // 3):
                if p >= n or m > 4096:
                    continue
                try:
                    pl = qpx.plan(n, m, p)
                except qpx.QPError:
                    continue  # beyond the supported sizes
                assert pl["lds_bytes"] + STATIC_LDS <= 160 * 1024, (n, m, p, pl)
