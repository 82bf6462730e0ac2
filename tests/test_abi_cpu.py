"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point that include/*.h declares, and validates arguments."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_15217_amd", "liblupp.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2609_15217_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def declared_functions():
    names = set()
    for h in ("lupp.h",):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", text,
                             flags=re.M):
            name = m.group(1)
            if name not in ("if", "sizeof", "defined"):
                names.add(name)
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lupp_create", "lupp_destroy", "lupp_batched_solve", "lupp_batched_solve_ragged",
                 "constitutive_update", "lupp_check_solve_args", "lupp_error_string"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = sorted(declared_functions() - exported)
    assert not missing, missing
    for name in declared_functions():
        getattr(lib, name)


def test_binding_names_match_the_header():
    import paper_2609_15217_amd.lupp as L
    for name in declared_functions():
        assert hasattr(L, name), name


def test_argument_validation_without_device():
    import paper_2609_15217_amd.lupp as L
    P = 0x1000  # never dereferenced: validation only
    ok = dict(n=8, batch=10, layout=L.LUPP_AOS, A=P, lda=8, strideA=64, b=P, strideB=8, ipiv=P,
              info=P, flags=0)

    def chk(**kw):
        a = dict(ok, **kw)
        return L.lupp_check_solve_args(a["n"], a["batch"], a["layout"], a["A"], a["lda"],
                                       a["strideA"], a["b"], a["strideB"], a["ipiv"], a["info"],
                                       a["flags"])

    assert chk() == 0
    assert chk(n=0) == -2 and chk(n=33) == -2
    assert chk(batch=-1) == -3
    assert chk(layout=2) == -4
    assert chk(A=None) == -5
    assert chk(lda=7) == -6
    assert chk(strideA=63) == -7
    assert chk(b=None) == -8
    assert chk(strideB=7) == -9
    assert chk(ipiv=None) == -10
    assert chk(info=None) == -11
    assert chk(flags=8) == -12
    # batch 0 accepts null buffers
    assert chk(batch=0, A=None, b=None, ipiv=None, info=None) == 0
    # SoA: the batch stride must cover the batch
    assert chk(layout=L.LUPP_SOA, strideA=10, strideB=10) == 0
    assert chk(layout=L.LUPP_SOA, strideA=9, strideB=10) == -7
    assert chk(layout=L.LUPP_SOA, strideA=10, strideB=9) == -9
    assert L.lupp_error_string(-7) == "argument 7 is invalid"
    assert "not supported" in L.lupp_error_string(L.LUPP_E_UNSUPPORTED)


def test_null_context_rejected():
    import paper_2609_15217_amd.lupp as L

    class Fake:
        handle = ctypes.c_void_p(0)

    rc = L.lupp_batched_solve(Fake(), 8, 1, 0, 0x1000, 8, 64, 0x1000, 8, 0x1000, 0x1000, 0, 0)
    assert rc == -1


def test_ragged_lane_counts_without_device():
    """The lane counts the ragged kernels hold for each size: every size has
    the thread path or a segment width, the default table's choice among them,
    and nothing beyond 32 lanes or outside 1..32."""
    import paper_2609_15217_amd.lupp as L

    class Fake:
        handle = ctypes.c_void_p(0)

    for n in range(1, 33):
        ok = [t for t in (1, 2, 4, 8, 16, 32, 64) if L.lupp_ragged_lanes_supported(n, t)]
        assert ok, n
        assert 64 not in ok
        # a segment never has more lanes than twice the rows it needs
        assert all(t == 1 or t < 2 * n for t in ok), (n, ok)
        if n > 16:
            assert ok == [16]
        default = 1 if n <= 5 else (8 if n <= 16 else 16)
        assert default in ok
    assert L.lupp_ragged_lanes_supported(0, 1) == 0
    assert L.lupp_ragged_lanes_supported(33, 16) == 0
    assert L.lupp_set_ragged_lanes(Fake(), 8, 8) == -1
    assert L.lupp_get_ragged_lanes(Fake(), 8) == -1
    assert L.lupp_autotune_ragged(Fake(), 8, 10, 0x1000, 0x1000, stream=0)[0] == -1
