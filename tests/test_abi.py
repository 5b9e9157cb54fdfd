"""The C ABI library loads without a GPU and exports every function that
include/f3r.h declares (no compute call is made here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "f3r.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(f3r_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("f3r_setup", "f3r_solve", "f3r_fgmres_solve", "f3r_get_history",
                 "f3r_get_weights", "f3r_set_weights", "f3r_params_default", "f3r_destroy",
                 "f3r_status_str", "f3r_setup_batched", "f3r_solve_batched",
                 "f3r_batch_get_history", "f3r_batch_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2505_20719_amd import f3r as B
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert set(B.EXPORTS) == set(declared_functions())


def test_host_only_calls_without_gpu():
    import paper_2505_20719_amd as P
    p = P.params_default(P.VARIANT_FP16)
    assert p.nlev == 4 and [p.lev[d].m for d in range(4)] == [100, 8, 4, 2] and p.c == 64
    assert [p.lev[d].prec_a for d in range(4)] == [P.FP64, P.FP32, P.FP16, P.FP16]
    assert [p.lev[d].prec_v for d in range(4)] == [P.FP64, P.FP32, P.FP32, P.FP16]
    q = P.params_default(P.VARIANT_FGMRES64)
    assert q.nlev == 1 and q.lev[0].m == 64
    assert P.lib().f3r_status_str(P.ERR_RANGE) == b"value out of range of a narrow format"
