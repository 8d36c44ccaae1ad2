"""The C-ABI library loads and exports every symbol the header declares (no
GPU needed: nothing here launches work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "jfnk.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jfnk_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libjfnk():
    from paper_1904_08510_amd import jfnk
    if not os.path.exists(jfnk.LIB_PATH):
        from paper_1904_08510_amd import build_ext
        build_ext.build()
    return jfnk


def test_library_exports_every_declared_symbol(libjfnk):
    names = header_functions()
    assert "jfnk_step" in names and "jfnk_create" in names
    L = ctypes.CDLL(libjfnk.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name
    assert set(libjfnk.EXPORTED_SYMBOLS) == set(names)


def test_config_defaults(libjfnk):
    cfg = libjfnk.default_config()
    assert cfg.gmres_restart == 30 and cfg.max_newton == 50 and cfg.tol_f == 1e-10
    assert cfg.gamma == 1e-4 and cfg.prec_precision == libjfnk.PREC_FP32
    assert cfg.ls_theta == 0.25 and cfg.chord_tol == 1e-3 and cfg.tol_x == 1e-10
    ncfg = libjfnk.net_default_config()
    assert ncfg.max_cols == 0 and abs(ncfg.out_scale_ne - 0.1) < 1e-7 and abs(ncfg.beta2 - 0.999) < 1e-7


def test_create_rejects_bad_config_without_touching_a_device(libjfnk):
    L = libjfnk.lib()
    h = ctypes.c_void_p()
    for kw in (dict(gmres_restart=31), dict(gmres_restart=0), dict(tol_f=0.0), dict(gamma=1.5),
               dict(max_cols=0), dict(threads_override=100), dict(schedule=7), dict(chord_tol=-1.0),
               dict(chord_tol=1.0), dict(ls_theta=1.0)):
        cfg = libjfnk.default_config(**kw)
        assert L.jfnk_create(ctypes.byref(cfg), ctypes.byref(h)) == libjfnk.JFNK_EINVAL
        assert not h.value
    assert L.jfnk_create(None, ctypes.byref(h)) == libjfnk.JFNK_EINVAL


def test_null_safety(libjfnk):
    L = libjfnk.lib()
    L.jfnk_destroy(None)
    assert L.jfnk_last_error(None) == b"null context"
    assert L.jfnk_step(None, None, None, None, None) == libjfnk.JFNK_EINVAL


def test_net_create_rejects_bad_config_without_touching_a_device(libjfnk):
    L = libjfnk.lib()
    h = ctypes.c_void_p()
    for kw in (dict(max_cols=4), dict(max_total_cells=100), dict(out_scale_ne=0.0), dict(beta1=1.0),
               dict(adam_eps=0.0), dict(max_cols=-1, max_total_cells=-1)):
        cfg = libjfnk.net_default_config(**kw)
        assert L.jfnk_net_create(ctypes.byref(cfg), ctypes.byref(h)) == libjfnk.JFNK_EINVAL
        assert not h.value
    assert L.jfnk_net_param_count() == 85442
    L.jfnk_net_destroy(None)
    assert L.jfnk_net_last_error(None) == b"null network"


def test_build_targets_gfx950_without_packed_fp32():
    """Every HIP source of the package is compiled, for gfx950 alone, with the
    packed-FP32 instructions turned off for the device code."""
    from paper_1904_08510_amd import build_ext
    f = build_ext.HIPCC_FLAGS
    assert "--offload-arch=gfx950" in f
    assert not any(x.startswith("--offload-arch=") and x != "--offload-arch=gfx950" for x in f)
    i = f.index("-packed-fp32-ops")
    assert f[i - 3:i] == ["-Xclang", "-target-feature", "-Xclang"]
    srcs = sorted(os.listdir(os.path.join(ROOT, "paper_1904_08510_amd", "csrc")))
    assert sorted(s for s in srcs if s.endswith(".hip")) == sorted(build_ext.SOURCES)


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the bindings raise: there is no other
    implementation to fall back to.  Run in a fresh interpreter so that an
    already loaded library does not answer."""
    import subprocess
    import sys
    code = (
        "import paper_1904_08510_amd.jfnk as J\n"
        f"J.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
        "try:\n"
        "    J.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "else:\n"
        "    print('loaded')\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("raised: libjfnk.so not built"), out.stdout
