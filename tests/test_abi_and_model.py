"""Host-only checks: the C ABI library loads and exports what include/lqs.h
declares, argument validation answers without a GPU, ctypes structs match the
C layout, and the roofline model reproduces the paper's printed numbers."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqs.h")
LIBPATH = os.path.join(ROOT, "paper_2502_03249_amd", "liblqs.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^(?:lqs_status|void|const char \*)\s*\*?(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIBPATH):
        from paper_2502_03249_amd import build
        build.build()
    return ctypes.CDLL(LIBPATH)


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert {"dslash_apply", "dslash_dagger", "cg_solve", "fermion_force"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_the_header(L):
    import paper_2502_03249_amd as lqs
    assert set(_declared()) == set(lqs.EXPORTS)


def test_field_bytes_and_validation(L):
    f = L.lqs_field_bytes
    f.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    f.restype = ctypes.c_int32
    n = ctypes.c_size_t()
    dims = (ctypes.c_int32 * 4)(4, 6, 8, 10)
    assert f(dims, 0, 2, ctypes.byref(n)) == 0 and n.value == 48 * 960 * 2
    assert f(dims, 1, 1, ctypes.byref(n)) == 0 and n.value == 24 * 960
    assert f(dims, 2, 3, ctypes.byref(n)) == 0 and n.value == 16 * 960 * 3
    assert f((ctypes.c_int32 * 4)(4, 5, 8, 10), 0, 1, ctypes.byref(n)) == -1
    assert f(dims, 0, 17, ctypes.byref(n)) == -1
    assert f(dims, 0, 0, ctypes.byref(n)) == -1
    assert f(dims, 2, 16, ctypes.byref(n)) == 0 and n.value == 16 * 960 * 16
    assert f(dims, 3, 1, ctypes.byref(n)) == -1
    L.lqs_strerror.restype = ctypes.c_char_p
    assert L.lqs_strerror(-4).decode().startswith("CG breakdown")


def test_null_handles_rejected_before_any_launch(L):
    for name in ("dslash_apply", "dslash_dagger"):
        fn = getattr(L, name)
        fn.restype = ctypes.c_int32
        assert fn(None, None, 18, None, None, None) == -1
    L.cg_solve.restype = ctypes.c_int32
    assert L.cg_solve(None, 1, None, None, None, None) == -1
    L.fermion_force.restype = ctypes.c_int32
    assert L.fermion_force(None, None, None, None, ctypes.c_double(1.0), 0, None, None) == -1
    L.lqs_last_error.restype = ctypes.c_char_p
    assert b"NULL" in L.lqs_last_error()
    for name, args in (("gauge_action", (None, None, None, ctypes.c_double(1.0), None, None)),
                       ("kinetic_energy", (None, None, None, None, None)),
                       ("hmc_trajectory", (None, None, None, None, None, ctypes.c_double(0.5), None, None, None,
                                           None, None))):
        fn = getattr(L, name)
        fn.restype = ctypes.c_int32
        assert fn(*args) == -1


def test_ctypes_structs_match_c_layout(tmp_path):
    import paper_2502_03249_amd as lqs
    src = tmp_path / "sz.c"
    src.write_text('#include "lqs.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lqs_field), sizeof(lqs_problem), '
                   'sizeof(lqs_cg_params), sizeof(lqs_cg_stats), offsetof(lqs_cg_params, reliable_delta), '
                   'offsetof(lqs_cg_stats, true_rel_residual), sizeof(lqs_hmc_params), sizeof(lqs_hmc_stats), '
                   'offsetof(lqs_hmc_params, cg), offsetof(lqs_hmc_stats, plaquette), '
                   'offsetof(lqs_hmc_params, fermions), offsetof(lqs_hmc_params, force_tol));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(lqs.LqsField), ctypes.sizeof(lqs.LqsProblem), ctypes.sizeof(lqs.LqsCgParams),
            ctypes.sizeof(lqs.LqsCgStats), lqs.LqsCgParams.reliable_delta.offset,
            lqs.LqsCgStats.true_rel_residual.offset, ctypes.sizeof(lqs.LqsHmcParams), ctypes.sizeof(lqs.LqsHmcStats),
            lqs.LqsHmcParams.cg.offset, lqs.LqsHmcStats.plaquette.offset, lqs.LqsHmcParams.fermions.offset,
            lqs.LqsHmcParams.force_tol.offset]
    assert got == want


def _golden():
    out = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_roofline.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_model_reproduces_paper_numbers():
    """Sec. 4.3: 570 flop/site, 126 floats/site, AI 0.57 (FP64) and 1.13 (FP32)."""
    from paper_2502_03249_amd import model
    gold = _golden()
    assert model.FLOPS_PER_SITE == gold["flops_per_site"]
    lps, rec = int(gold["links_per_site_paper"]), int(gold["reals_per_link_paper"])
    assert model.hop_model_bytes(model.F64, rec, 1, lps) / 8 == gold["floats_per_site_paper"]
    assert round(model.arithmetic_intensity(model.F64, rec, 1, lps), 2) == gold["ai_fp64"]
    assert round(model.arithmetic_intensity(model.F32, rec, 1, lps), 2) == gold["ai_fp32"]
    # the printed multi-vector formula n*570/(8*(6*12 + n*(9*6))) for FP64
    for n in (1, 2, 4, 8, 16):
        assert abs(model.arithmetic_intensity(model.F64, 12, n, 6) - n * 570 / (8 * (6 * 12 + n * 9 * 6))) < 1e-15


def test_model_bytes_of_the_formats():
    from paper_2502_03249_amd import model
    assert model.hop_model_bytes(model.F64) == 1584 and model.hop_model_bytes(model.F64, 12) == 1200
    assert model.hop_model_bytes(model.F32) == 792 and model.hop_model_bytes(model.F32, 12) == 600
    assert model.hop_model_bytes(model.F16) == 432 and model.hop_model_bytes(model.F16, 12) == 336
    assert model.hop_min_bytes(model.F64) == 1248
