"""The C-ABI library loads and exports every symbol include/m1.h declares, its
structs match the binding, and host-side validation rejects bad configurations
before touching a GPU.  CPU only."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "m1.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(m1_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported():
    import paper_2011_13926_amd as P
    lib = ctypes.CDLL(P.LIB_PATH)
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) <= set(P.EXPORTED)


def test_struct_sizes_match():
    import paper_2011_13926_amd as P
    assert P._lib.m1_config_size() == ctypes.sizeof(P.M1Config)
    assert P._lib.m1_stats_size() == ctypes.sizeof(P.M1Stats)


def _setup(cfg, fields=None):
    import paper_2011_13926_amd as P
    ctx = ctypes.c_void_p()
    st = P.m1_setup(ctypes.byref(cfg), ctypes.byref(fields) if fields is not None else None, None, None, 1.0,
                    None, ctypes.byref(ctx))
    return st, P.m1_last_error(None).decode(), ctx


@pytest.mark.parametrize("field,value,msg", [
    ("ndim", 4, "ndim"), ("dx", -1.0, "dx"), ("restart", 0, "restart"), ("restart", 49, "restart"),
    ("source", 7, "enum"), ("rtol", float("nan"), "tolerances"), ("lambda_floor", -0.1, "lambda_floor"),
])
def test_invalid_config_rejected_on_host(field, value, msg):
    import paper_2011_13926_amd as P
    import workloads as W
    p = W.random_problem((4, 4), 0)
    cfg = P.make_config(p)
    setattr(cfg, field, value)
    st, err, ctx = _setup(cfg)
    assert st == P.M1_ERR_INVALID_ARG
    assert msg in err
    assert not ctx.value


def test_periodic_pairing_and_missing_fields():
    import paper_2011_13926_amd as P
    import workloads as W
    p = W.random_problem((4, 4), 0)
    cfg = P.make_config(p)
    cfg.bc[0] = P.BC["outflow"]          # -x outflow, +x periodic: inconsistent
    st, err, _ = _setup(cfg)
    assert st == P.M1_ERR_INVALID_ARG and "periodic" in err
    cfg = P.make_config(p)
    st, err, _ = _setup(cfg, P.M1Fields())   # sigma NULL
    assert st == P.M1_ERR_INVALID_ARG and "sigma" in err
    q = W.random_problem((4, 4), 0, bc=["dirichlet", "outflow", "periodic", "periodic"])
    cfg = P.make_config(q)
    f = P.M1Fields()
    f.sigma = 1234                            # never dereferenced: validation fails first
    st, err, _ = _setup(cfg, f)
    assert st == P.M1_ERR_INVALID_ARG and "Dirichlet" in err


def test_status_strings():
    import paper_2011_13926_amd as P
    assert P.m1_status_string(P.M1_NOT_CONVERGED) == b"M1_NOT_CONVERGED"
    assert P.m1_status_string(P.M1_ERR_NONFINITE) == b"M1_ERR_NONFINITE"
    assert "arnoldi_update" in P.kernel_classes()
