"""CPU checks of the C ABI: the library loads, exports every function
include/ssm.h declares, and rejects invalid configurations before touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2105_09688_amd import _lib, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "ssm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssm_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_functions():
    assert set(_header_functions()) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _header_functions():
        assert hasattr(lib, name), name


def _c_layout(tmp_path, struct, fields):
    """sizeof/offsetof of a struct of include/ssm.h, as the C compiler lays it out."""
    import subprocess
    src = tmp_path / "layout.c"
    body = "".join(f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ssm.h"\n'
                   f'int main(void){{printf("%zu\\n", sizeof({struct}));{body}return 0;}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("struct,cls", [("ssm_config", _lib.Config), ("ssm_info_t", _lib.Info), ("ssm_train_cfg", _lib.TrainCfg),
                                        ("ssm_surrogate_train_cfg", _lib.SurrTrainCfg)])
def test_struct_layout_matches_header(tmp_path, struct, cls):
    names = [f for f, _ in cls._fields_]
    got = _c_layout(tmp_path, struct, names)
    assert got[0] == C.sizeof(cls)
    assert got[1:] == [getattr(cls, f).offset for f in names]


def _init(w, **over):
    lib = _lib.load()
    from paper_2105_09688_amd.ssm import PRECISIONS
    d = w["d"]
    n = len(w["systems"])
    Ns = (C.c_int64 * n)(*[s[0] for s in w["systems"]])
    ens = (C.c_int32 * n)(*[s[1] for s in w["systems"]])
    hs = (C.c_double * n)(*[s[2] for s in w["systems"]])
    c = _lib.Config()
    c.d, c.n_sys, c.N, c.ens, c.h = d, n, Ns, ens, hs
    c.T, c.h_fine, c.seed, c.precision = w["T"], w["h_fine"], 0, PRECISIONS["fp64"]
    c.v_rho, c.v_a = w["v"].get("rho", 0.0), w["v"].get("a", 0.0)
    c.b_g, c.b_ell = w["b"].get("g", 0.0), w["b"].get("ell", 1.0)
    for k, v in over.items():
        setattr(c, k, v)
    h = C.c_void_p()
    st = lib.ssm_init(C.byref(c), C.byref(h))
    return st, lib.ssm_last_error().decode()


@pytest.mark.parametrize("field,value,needle", [
    ("d", 0, "d must be"),
    ("d", 5, "d must be"),
    ("T", -1.0, "T must be"),
    ("h_fine", 0.0, "h_fine"),
    ("v_a", -1.0, "v_a"),
    ("b_ell", 0.0, "b_ell"),
    ("precision", 7, "precision"),
    ("targets_per_lane", 3, "targets_per_lane"),
    ("sources_per_item", 10, "sources_per_item"),
    ("kahan_span", 2, "kahan_span"),
    ("kahan_span", 1, "FP32-compensated"),  # the helper's precision is FP64
])
def test_init_rejects_invalid_config(field, value, needle):
    st, msg = _init(W.small_parity(n_ens=1, N=10), **{field: value})
    assert st == _lib.SSM_ERR_INVALID and needle in msg, msg


def test_per_pair_compensation_runs_ordered_pairs_only():
    st, msg = _init(W.small_parity(n_ens=1, N=10), precision=_lib.SSM_FP32_KAHAN, kahan_span=1, pair_scheme=2)
    assert st == _lib.SSM_ERR_INVALID and "ordered" in msg, msg


def test_init_rejects_non_integer_grid_and_step_constraint():
    w = W.small_parity(n_ens=1, N=10, h=0.3)  # T/h not an integer
    st, msg = _init(w)
    assert st == _lib.SSM_ERR_INVALID and "T / h" in msg
    w = W.small_parity(n_ens=1, N=10, h=2.0 ** -8, h_fine=3e-4)  # h/h_fine not an integer
    st, msg = _init(w)
    assert st == _lib.SSM_ERR_INVALID and "h_fine" in msg
    w = W.ou(rho=6.0, h=2.0 ** -3, T=0.25)  # Theorem 2.6: 1 - h(2 rho + 1) <= 0
    st, msg = _init(w)
    assert st == _lib.SSM_ERR_INVALID and "Theorem 2.6" in msg
    w = W.ou(rho=10.0, h=2.0 ** -3, T=0.25)  # Lemma 4.1: 1 - h rho <= 0
    st, msg = _init(w, allow_unstable_h=1)
    assert st == _lib.SSM_ERR_INVALID and "Lemma 4.1" in msg


def test_init_rejects_incommensurate_levels():
    w = W.small_parity(n_ens=1, N=10)
    w["systems"] = [(10, 0, 2.0 ** -4), (10, 0, 3 * 2.0 ** -8)]
    w["h_fine"] = 2.0 ** -8
    st, msg = _init(w)
    assert st == _lib.SSM_ERR_INVALID


def test_init_rejects_empty_and_degenerate_inputs():
    """Empty systems, no systems, a non-finite horizon or step, and a
    component-wise cubic of the wrong sign are refused on the host."""
    w = W.small_parity(n_ens=1, N=10)
    w["systems"] = [(0, 0, 2.0 ** -8)]
    st, msg = _init(w)
    assert st == _lib.SSM_ERR_INVALID and "N out of range" in msg
    st, msg = _init(W.small_parity(n_ens=1, N=10), n_sys=0)
    assert st == _lib.SSM_ERR_INVALID
    st, msg = _init(W.small_parity(n_ens=1, N=10), T=float("nan"))
    assert st == _lib.SSM_ERR_INVALID and "T must be" in msg
    w = W.small_parity(n_ens=1, N=10)
    w["systems"] = [(10, 0, float("inf"))]
    st, msg = _init(w)
    assert st == _lib.SSM_ERR_INVALID
    c_ak = (C.c_double * 4)(-1.0, 0.0, 0.0, 0.0)
    st, msg = _init(W.small_parity(n_ens=1, N=10), v_componentwise=1, v_ak=c_ak)
    assert st == _lib.SSM_ERR_INVALID and "v_ak" in msg


def test_kernel_level_entry_points_validate_on_host():
    lib = _lib.load()
    assert lib.ssm_pair_sum(0, 10, 0, None, 1.0, None, None, 0, None) == _lib.SSM_ERR_INVALID
    assert lib.ssm_pair_workspace_bytes(0, 10, 0) == 0
    assert lib.ssm_pair_workspace_bytes(1, 1000, 1) > 0
    assert lib.ssm_brownian(1, 10, 0, 0, 0, 0, 1e-3, None, None) == _lib.SSM_ERR_INVALID
    assert lib.ssm_philox_blocks(0, 0, 0, 0, 0, 0, 0, None, None) == _lib.SSM_ERR_INVALID


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle, and refuses to run without libssm."""
    import paper_2105_09688_amd
    pkg = os.path.dirname(paper_2105_09688_amd.__file__)
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
