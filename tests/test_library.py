"""Host-only checks of the C-ABI library: it is built for gfx950, loads, and exports exactly
the entry points include/thc.h declares; the binding and the library refuse bad arguments; the
working-memory planner's plans (no GPU call is made)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "thc.h")
LIB = os.path.join(ROOT, "paper_2111_11473_amd", "libthc.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(thc_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libthc.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_binding_symbols():
    from paper_2111_11473_amd import thc
    assert _declared() == sorted(thc.SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (thc_[a-z_0-9]+)$", out, flags=re.M))
    assert exported == set(_declared())


def test_library_contains_gfx950_code():
    """The device code object bundled in the library targets gfx950 (MI355X)."""
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_binding_refuses_host_tensors():
    import torch
    from paper_2111_11473_amd import thc
    with pytest.raises(TypeError):
        thc._ptr(torch.zeros(3, dtype=torch.float64))


def test_binding_fails_loudly_without_the_library(tmp_path):
    """With no built library there is no fallback: loading it raises ImportError naming the build
    step (in a fresh interpreter, since a loaded library is kept for the process)."""
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2111_11473_amd import thc\n"
            "try:\n    thc.load(%r)\nexcept ImportError as e:\n    print('ImportError', e)\n") % (
                ROOT, str(tmp_path / "libthc.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ImportError") and "build" in r.stdout


@pytest.mark.parametrize("a,b,c,tA,tB", [
    ((4, 5), (6, 7), (4, 7), False, False),     # K of A and B differ
    ((4, 5), (5, 7), (4, 8), False, False),     # C too wide
    ((5, 4), (5, 7), (5, 7), True, False),      # op(A) has 4 rows, C 5
    ((4, 5), (5, 7), (4, 7), False, True),      # op(B) is 7 x 5
    ((2, 4, 5), (3, 5, 7), (2, 4, 7), False, False),  # B batch neither 1 nor C's
    ((4, 5), (1, 5, 7), (4, 7), False, False),  # mixed 2-D and 3-D
])
def test_dgemm_binding_checks_shapes(a, b, c, tA, tB):
    """Operand shapes that do not match are refused before any pointer reaches the library (the C
    entry point takes sizes and leading dimensions only and cannot check buffer lengths)."""
    import torch
    from paper_2111_11473_amd import thc
    z = lambda s: torch.zeros(s, dtype=torch.float64)
    with pytest.raises(ValueError):
        thc.dgemm(z(a), z(b), z(c), transA=tA, transB=tB)


@pytest.mark.parametrize("field,value", [("o", 0), ("v", -1), ("nL", 0), ("nP", 0), ("nQ", 0),
                                         ("nP", 10 * 40 + 1), ("nQ", 10 * 40 + 1), ("precision", 3),
                                         ("diis_max", 17), ("flags", 1 << 6), ("x_block", -64),
                                         ("split_mask", 1 << 6), ("guess", 2)])
def test_create_rejects_invalid_options(lib, field, value):
    """Option validation happens before any device call: sizes below 1, a pair basis or ERI grid
    larger than the o v pairs (singular metric / Gram matrix), out-of-range options."""
    from paper_2111_11473_amd import thc
    base = dict(o=10, v=40, nL=150, nP=120, nQ=300, singles=1, diis_max=8, tol_energy=1e-8, a_block=0,
                i_chunk=0, x_block=0, x_chunk=0, precision=0, flags=0, x7_chunk=0, q_pairs=0, q_jchunk=0,
                split_mask=0, guess=0, reserved=0)
    base[field] = value
    opt = thc.Options(**base)
    lib.thc_create.argtypes = [ctypes.POINTER(thc.Options), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    assert lib.thc_create(ctypes.byref(opt), None, ctypes.byref(h)) == -1  # THC_EINVAL
    assert not h.value


def test_memory_plans_of_the_workloads():
    """The working-memory planner (host only): the fp64 workload (o=50 v=450 nL=1500 nP=1000
    nQ=2500) runs as one H block and one Alg. 7 chunk in ~41 GB; the mixed-precision workload
    (o=200 v=1800 nL=6000 nP=4000 nQ=10000, synthetic inputs) fits 270 GB with the vv Cholesky block
    regenerated per fused-pass block, H blocks of 512 ranks with 256-point grid chunks and Alg. 7 in
    row chunks; the ~2500-basis-function workload (o=350 v=2150 nL=10000 nP=7000 nQ=17500) does not
    fit with FP64 intermediates (its B_ia^I alone is 105 GB)."""
    from paper_2111_11473_amd import synth, thc
    c = synth.CONFIGS["fp64"]
    p = thc.plan_query(c.o, c.v, c.nL, c.nP, c.nQ, 270e9)
    assert (p["x_blocks"], p["i_chunk"], p["x7_chunks"], p["lvv_resident"]) == (1, 638, 1, 1)
    assert 35e9 < p["device_bytes"] < 45e9
    c = synth.CONFIGS["mixed"]
    for prec in (0, 1):
        p = thc.plan_query(c.o, c.v, c.nL, c.nP, c.nQ, 270e9, synthetic=True, precision=prec)
        assert p["device_bytes"] <= 270e9 and p["lvv_resident"] == 0 and p["exchange_fused"] == 1
        assert p["x_block"] == 512 and p["i_chunk"] == 256 and p["x7_chunks"] > 1
    c = synth.CONFIGS["paper"]
    with pytest.raises(thc.ThcError, match="THC_ENOMEM"):
        thc.plan_query(c.o, c.v, c.nL, c.nP, c.nQ, 270e9, synthetic=True, precision=1)


def test_mixed_plan_shares_the_fp64_buffers():
    """The mixed path's FP32 E, F and G live in the FP64 buffers (a residual uses one precision or
    the other), so its plan walks the same grid-point chunks as the FP64 one; it only adds the
    FP32 H-kernel's tile table (a few bytes per tile)."""
    from paper_2111_11473_amd import synth, thc
    c = synth.CONFIGS["fp64"]
    p0 = thc.plan_query(c.o, c.v, c.nL, c.nP, c.nQ, 270e9, precision=0)
    p1 = thc.plan_query(c.o, c.v, c.nL, c.nP, c.nQ, 270e9, precision=1)
    assert (p1["i_chunk"], p1["x_block"], p1["x7_chunk"]) == (p0["i_chunk"], p0["x_block"], p0["x7_chunk"])
    assert 0 <= p1["device_bytes"] - p0["device_bytes"] <= 4 * 2 * p0["h_tiles"] + 64 * 1024 * 1024


def test_planner_properties_over_random_sizes():
    """The working-memory planner over 600 seeded random problems, budgets from 0.1 to 270 GB,
    both precisions, caller or synthetic inputs and either Alg. 6 or Alg. 4-5: every plan it
    returns needs no more than its budget; planning again for exactly the bytes it reported
    succeeds within them (what a caller's workspace of that size relies on); every block and chunk
    is within its loop's range; the H-kernel table holds every (Y <= Z) block pair and Z slice of
    each X tile in whole generations; anything else is THC_ENOMEM."""
    import random
    from paper_2111_11473_amd import thc
    rng = random.Random(7)
    fitted = 0
    for _ in range(600):
        o = rng.choice([1, 2, 5, 10, 30, 50, 80, 120, 200, 350])
        v = max(1, int(o * rng.uniform(1, 12)))
        nL = max(1, int((o + v) * rng.uniform(0.5, 4)))
        nP = max(1, min(o * v, int(rng.uniform(0.2, 25) * o)))
        nQ = max(1, min(o * v, int(nP * rng.uniform(1, 3))))
        budget = 10 ** rng.uniform(8, 11.43)
        kw = dict(synthetic=rng.random() < 0.5, precision=rng.choice([0, 1]),
                  flags=rng.choice([0, 0, thc.FLAG_QUARTIC, thc.FLAG_QUINTIC]))
        try:
            p = thc.plan_query(o, v, nL, nP, nQ, budget, **kw)
        except thc.ThcError as e:
            assert e.rc == thc.THC_ENOMEM, e
            continue
        fitted += 1
        case = (o, v, nL, nP, nQ, budget, kw)
        assert 0 < p["device_bytes"] <= budget, case
        again = thc.plan_query(o, v, nL, nP, nQ, p["device_bytes"], **kw)
        assert again["device_bytes"] <= p["device_bytes"], case
        assert 1 <= p["a_block"] <= nL and p["alg1_tile"] in (64, 128) and 1 <= p["alg1_splits"] <= 16, case
        assert 1 <= p["x_chunk"] <= nP and 1 <= p["x7_chunk"] <= nP, case
        assert p["exchange_fused"] == int(o <= 200), case
        assert p["lvv_resident"] == 1 or kw["synthetic"], case
        if p["quintic"]:
            assert kw["flags"] != thc.FLAG_QUARTIC, case
            assert 1 <= p["q_jchunk"] <= o and 1 <= p["q_pairs"] <= max(o, v), case
        else:
            assert kw["flags"] != thc.FLAG_QUINTIC, case
            p64, nB = -(-nP // 64) * 64, -(-nP // 16)
            assert p["x_block"] % 64 == 0 and 64 <= p["x_block"] <= p64, case
            assert 1 <= p["i_chunk"] <= nQ, case
            assert p["h_tiles"] == nB * (nB + 1) // 2 * 2 * (p["x_block"] // 64), case
            assert 0 <= p["h_generations"] * 8 * 64 - p["h_tiles"] < 8 * 64, case
    assert fitted > 300


def test_binding_matches_the_c_header(tmp_path):
    """The binding's ctypes structures have the C header's layout (every field's offset and size,
    and each structure's size), and its constants equal the header's #defines -- checked by a C
    program compiled against include/thc.h as strict C99 (the header is plain C)."""
    import shutil
    from paper_2111_11473_amd import thc
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    structs = {"thc_options": thc.Options, "thc_plan_info": thc.PlanInfo, "thc_synth_spec": thc.SynthSpec}
    names = re.findall(r"^#define (THC_[A-Z_0-9]+)[ \t]+\S", open(HEADER).read(), flags=re.M)
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "thc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("size {cname} %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("field {cname}.{field} %zu %zu\\n", offsetof({cname}, {field}), '
                         f'sizeof((({cname}*)0)->{field}));')
    for n in names:
        lines.append(f'  printf("const {n} %lld\\n", (long long)({n}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    r = subprocess.run([gcc, "-std=c99", "-pedantic", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    seen_consts = 0
    for line in filter(None, out):
        kind, what, *vals = line.split()
        if kind == "size":
            assert int(vals[0]) == ctypes.sizeof(structs[what]), line
        elif kind == "field":
            cname, field = what.split(".")
            desc = getattr(structs[cname], field)
            assert (int(vals[0]), int(vals[1])) == (desc.offset, desc.size), line
        else:
            py = what[4:] if not what.startswith(("THC_O", "THC_E")) else what  # THC_TERM_EQ28 -> TERM_EQ28
            if hasattr(thc, py):
                assert getattr(thc, py) == int(vals[0]), line
                seen_consts += 1
    assert seen_consts == len(names)


def test_binding_prototypes_match_the_c_header():
    """Every function of include/thc.h is declared to ctypes with the header's argument list:
    the same number of arguments, pointers where the header has pointers, and the same integer
    width and signedness or floating type for each scalar."""
    import ctypes as C
    from paper_2111_11473_amd import thc
    lib = thc.load()
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    scalars = {"int64_t": C.c_int64, "int32_t": C.c_int32, "int": C.c_int, "uint32_t": C.c_uint32,
               "uint64_t": C.c_uint64, "double": C.c_double, "float": C.c_float, "size_t": C.c_size_t}
    protos = re.findall(r"\b(?:int|void|const char\s*\*)\s*(thc_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", txt)
    assert {p[0] for p in protos} == set(_declared())
    for name, args in protos:
        params = [a.strip() for a in args.split(",") if a.strip() and a.strip() != "void"]
        declared = getattr(lib, name).argtypes
        assert declared is not None and len(declared) == len(params), (name, params, declared)
        for p, t in zip(params, declared):
            if "*" in p:
                assert t in (C.c_void_p, C.c_char_p) or issubclass(t, C._Pointer), (name, p, t)
            else:
                ctype = " ".join(p.split()[:-1]).replace("const ", "")
                want = scalars[ctype]
                assert C.sizeof(t) == C.sizeof(want) and t(-1).value == want(-1).value, (name, p, t)
                assert isinstance(t(0).value, float) == isinstance(want(0).value, float), (name, p, t)


@pytest.mark.parametrize("case", ["lda", "ldb", "ldc", "ldaT", "ldbT", "nullA", "nullB", "nullC", "negK", "negStride"])
def test_dgemm_entry_point_refuses_bad_arguments(lib, case):
    """thc_dgemm refuses, before any launch, operands it could not address: a leading dimension
    shorter than a row of op(A), op(B) or C, a missing operand, negative sizes or strides.  Run only
    where there is no GPU: the operands are placeholder addresses, so a regression that let one of
    these calls through must not reach a device."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("placeholder operand addresses are only passed where no GPU exists")
    from paper_2111_11473_amd import thc
    f = thc.load().thc_dgemm
    a = dict(tA=0, tB=0, M=4, N=5, K=6, lda=6, ldb=5, ldc=5, sA=0, sB=0, sC=0, A=1, B=1, C=1)
    a.update({"lda": dict(lda=5), "ldb": dict(ldb=4), "ldc": dict(ldc=4), "ldaT": dict(tA=1, lda=3),
              "ldbT": dict(tB=1, ldb=5), "nullA": dict(A=0), "nullB": dict(B=0), "nullC": dict(C=0),
              "negK": dict(K=-1), "negStride": dict(sC=-1)}[case])
    p = lambda x: ctypes.c_void_p(0x10000 if x else None)
    rc = f(a["tA"], a["tB"], a["M"], a["N"], a["K"], 1.0, p(a["A"]), a["lda"], a["sA"], p(a["B"]), a["ldb"],
           a["sB"], 0.0, p(a["C"]), a["ldc"], a["sC"], 1, None)
    assert rc == thc.THC_EINVAL


def test_dgemm_entry_point_empty_product_is_a_no_op(lib):
    from paper_2111_11473_amd import thc
    f = thc.load().thc_dgemm
    for M, N, nb in ((0, 5, 1), (4, 0, 1), (4, 5, 0)):
        assert f(0, 0, M, N, 6, 1.0, None, 6, 0, None, 5, 0, 0.0, None, 5, 0, nb, None) == thc.THC_OK
