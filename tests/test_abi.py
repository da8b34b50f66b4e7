"""Host-side checks of the C ABI (no GPU needed, no compute call):
the library loads and exports every function include/lbm.h declares, the
binding's structs match the C layout, argument validation rejects bad
parameters before touching the device, and the product package does not
reach the oracle."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def lbm():
    import paper_1711_03254_amd.lbm as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1711_03254_amd import build
        build.build()
    m.load_library()
    return m


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("lbm_init", "lbm_step", "lbm_moments", "lbm_reduce", "lbm_get_populations",
              "lbm_set_populations", "lbm_set_fields", "lbm_info", "lbm_last_error", "lbm_free",
              "lbm_batch_create", "lbm_batch_step", "lbm_batch_last_error", "lbm_batch_free"):
        assert n in names


def test_library_exports_every_declared_symbol(lbm):
    lib = lbm.load_library()
    names = _declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(lbm.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lbm_\w+)", out))
    assert set(names) <= exported


def test_library_exports_the_surrogate_kernels(lbm):
    from paper_1711_03254_amd import nn
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "lbm_nn.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(nn_[a-z0-9_]+)\s*\(", text)))
    assert set(names) == set(nn.NN_EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert set(names) <= set(re.findall(r"\bT (nn_\w+)", out))
    nn.load()   # argument types bind to every symbol


def test_surrogate_calls_reject_bad_sizes_on_the_host(lbm):
    """Size and alignment checks happen before anything is enqueued (no
    device memory is touched: the pointers are never dereferenced)."""
    import ctypes
    from paper_1711_03254_amd import nn
    lib = nn.load()
    p = ctypes.c_void_p(1 << 20)
    assert lib.nn_conv3d_fwd(p, 16, p, None, p, 16, 1, 0, 1, 4, 4, 4, 8, 16, None) == lbm.LBM_EINVAL   # ci % 16
    assert lib.nn_conv3d_fwd(p, 18, p, None, p, 16, 1, 0, 1, 4, 4, 4, 16, 16, None) == lbm.LBM_EINVAL  # ldx % 4
    assert lib.nn_pool2_fwd(p, 16, p, 16, 1, 3, 4, 4, 16, None) == lbm.LBM_EINVAL                      # odd extent
    assert lib.nn_bwd_weight_work(1, 4, 4, 4, 16, 16) == 27 * 16 * 16
    assert lib.nn_conv3d_bwd_weight(p, 16, p, 16, p, p, p, 10, 1, 4, 4, 4, 16, 16, None) == lbm.LBM_EINVAL
    assert lib.nn_adam(p, p, p, p, None, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == lbm.LBM_EINVAL       # t < 1


def test_struct_layout_matches_c(lbm, tmp_path):
    prog = tmp_path / "layout.c"
    fields_p = [f for f, _ in lbm.lbm_params._fields_]
    fields_i = [f for f, _ in lbm.lbm_info_t._fields_]
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {",
             'printf("%zu %zu\\n", sizeof(lbm_params), sizeof(lbm_info_t));']
    for f in fields_p:
        lines.append(f'printf("p {f} %zu\\n", offsetof(lbm_params, {f}));')
    for f in fields_i:
        lines.append(f'printf("i {f} %zu\\n", offsetof(lbm_info_t, {f}));')
    lines += ["return 0; }"]
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sp, si = map(int, out[0].split())
    assert sp == ctypes.sizeof(lbm.lbm_params)
    assert si == ctypes.sizeof(lbm.lbm_info_t)
    for line in out[1:]:
        if not line:
            continue
        kind, name, off = line.split()
        cls = lbm.lbm_params if kind == "p" else lbm.lbm_info_t
        assert getattr(cls, name).offset == int(off), name


@pytest.mark.parametrize("bad,needle", [
    (dict(tau=(0.5, 1.0)), "tau"),
    (dict(tau=(1.0, 0.3)), "tau"),
    (dict(prec=7), "precision"),
    (dict(eq_kind=2), "eq_kind"),
    (dict(wall_kind=3), "wall_kind"),
    (dict(force_kind=-1), "force_kind"),
    (dict(tile=(48, 4)), "tile"),
    (dict(tile=(64, 8), prec=0), "256-thread"),
    (dict(tile=(32, 16), prec=0), "256-thread"),
    (dict(tile=(64, 16), prec=0), "256-thread"),
    (dict(nx=0), "dimensions"),
    (dict(check_every=-1), "check_every"),
    (dict(G=float("nan")), "finite"),
])
def test_init_rejects_bad_parameters_on_the_host(lbm, bad, needle):
    import numpy as np
    kw = dict(nx=4, ny=4, nz=4)
    kw.update({k: v for k, v in bad.items() if k in ("nx", "ny", "nz")})
    n = kw["nx"] * kw["ny"] * kw["nz"]
    r = np.ones(max(n, 1))
    p = lbm.Params(**kw, rho_init=(r, r), **{k: v for k, v in bad.items() if k not in ("nx", "ny", "nz")})
    with pytest.raises(lbm.LBMError) as ei:
        lbm.lbm_init(p)
    assert ei.value.code == lbm.LBM_EINVAL
    assert needle in str(ei.value)


def test_warm_start_calls_reject_null_arguments_on_the_host(lbm):
    """The restart, residual and distance entry points and the surrogate's
    feature / decoding kernels return LBM_EINVAL for NULL or bad arguments
    before any device work (no GPU needed)."""
    import ctypes
    from paper_1711_03254_amd import nn
    lib = nn.load()   # argument types of every call
    out = (ctypes.c_double * 2)()
    p = ctypes.c_void_p(8)
    assert lib.lbm_set_fields_strain(None, p, p, p, 0) == lbm.LBM_EINVAL
    assert lib.lbm_residual(None, out) == lbm.LBM_EINVAL
    assert lib.lbm_distance(None, p, p, 0, out) == lbm.LBM_EINVAL
    assert lib.nn_solid_distance(None, p, p, 4, 4, 4, 2, None) == lbm.LBM_EINVAL
    assert lib.nn_solid_distance(p, p, p, 4, 4, 4, 0, None) == lbm.LBM_EINVAL          # radius < 1
    assert lib.nn_features(p, p, p, p, ctypes.c_float(8.0), p, 16, 2, 64, None) == lbm.LBM_EINVAL   # c < 3
    assert lib.nn_features(p, p, p, p, ctypes.c_float(0.0), p, 16, 16, 64, None) == lbm.LBM_EINVAL  # scale
    dbl = ctypes.c_double
    assert lib.nn_decode_fields(p, 4, p, p, p, dbl(0.1), dbl(0.1), dbl(1e-5), ctypes.c_float(1.0),
                                ctypes.c_float(1.0), dbl(1e-3), p, p, p, p, 64, None) == lbm.LBM_EINVAL   # ldo < 5
    assert lib.nn_decode_fields(p, 16, p, p, p, dbl(0.0), dbl(0.1), dbl(1e-5), ctypes.c_float(1.0),
                                ctypes.c_float(1.0), dbl(1e-3), p, p, p, p, 64, None) == lbm.LBM_EINVAL   # nu_a
    with pytest.raises(lbm.LBMError):
        lbm.lbm_set_fields_strain(None, None, None, None)   # no velocity field


def test_init_rejects_oversized_plane(lbm):
    import numpy as np
    r = np.ones(1)
    with pytest.raises(lbm.LBMError) as ei:
        lbm.lbm_init(lbm.Params(2048, 2048, 512, prec=lbm.LBM_FP64, rho_init=(r, r)))
    assert ei.value.code == lbm.LBM_EINVAL and "too large" in str(ei.value)


def test_product_package_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_1711_03254_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, flags=re.M), f
                assert "liboracle" not in text and "oracle.c" not in text, f
