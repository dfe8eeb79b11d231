"""The C ABI library loads and exports every function include/perf_gn.h declares;
host-side argument validation (no GPU work is started by any call here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(perf_[A-Za-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2112_05598_amd import abi
    return abi.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_2112_05598_amd import abi
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert names == {s[0] for s in abi.SIGNATURES}


def test_binding_constants_match_the_header():
    """The binding's sizes are the header's #defines (the ABI's array sizes and row widths)."""
    from paper_2112_05598_amd import abi
    text = open(os.path.join(ROOT, "include", "perf_gn.h")).read()
    defs = dict(re.findall(r"#define[ \t]+(PERF_[A-Z0-9_]+)[ \t]+(.+)", text))
    assert len(defs) >= 5
    for name, expr in defs.items():
        assert getattr(abi, name) == eval(expr, {}), name


def _desc(**kw):
    import perf_synth as ps
    from paper_2112_05598_amd.scene import make_desc
    w = ps.workload("cfg1")
    d = make_desc(w.spec, 64, 64)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("field,value,msg", [
    ("nx", 1, "grid dims"),
    ("step_vox", 0.0, "step_vox"),
    ("step_vox", 1.5, "step_vox"),
    ("n_layers", 9, "n_layers"),
    ("env_w", 1, "env_w"),
    ("param_dtype", 7, "param_dtype"),
    ("width", 0, "image size"),
])
def test_descriptor_validation(lib, field, value, msg):
    d = _desc(**{field: value})
    assert lib.perf_workspace_bytes(ctypes.byref(d), 8) == 0
    assert msg in lib.perf_last_error().decode()


def test_layer_radius_must_enclose_box(lib):
    d = _desc()
    d.layer_radius[0] = 1.7  # box corner distance is sqrt(3) = 1.732
    assert lib.perf_workspace_bytes(ctypes.byref(d), 8) == 0
    assert "radius" in lib.perf_last_error().decode()
    d = _desc(n_layers=2)
    d.layer_radius[0], d.layer_radius[1] = 3.0, 2.0
    assert lib.perf_workspace_bytes(ctypes.byref(d), 8) == 0


def test_workspace_size_matches_layout(lib):
    d = _desc()
    n = lib.perf_workspace_bytes(ctypes.byref(d), 8)
    P = 4 * (32 ** 3 + 64 * 32)
    # six PCG vectors, blocks and the inverse blocks dominate
    assert n >= 4 * (6 * P + 5 * P // 4 + 10 * P // 4)
    d2 = _desc(param_dtype=1)
    assert lib.perf_workspace_bytes(ctypes.byref(d2), 8) >= n + 2 * P


def test_init_rejects_bad_arguments_before_device_work(lib):
    from paper_2112_05598_amd import abi
    from paper_2112_05598_amd.scene import make_cameras
    import perf_synth as ps
    w = ps.workload("cfg1")
    d = _desc()
    cams = make_cameras(w.cams)
    h = ctypes.c_void_p()
    n = lib.perf_workspace_bytes(ctypes.byref(d), 8)
    assert lib.perf_init_scene(ctypes.byref(d), cams, 8, None, None, n, None, ctypes.byref(h)) == abi.PERF_EINVAL
    assert lib.perf_init_scene(ctypes.byref(d), cams, 8, None, ctypes.c_void_p(4096 + 8), n, None,
                               ctypes.byref(h)) == abi.PERF_EINVAL
    assert "aligned" in lib.perf_last_error().decode()
    assert lib.perf_init_scene(ctypes.byref(d), cams, 8, None, ctypes.c_void_p(4096), n - 1, None,
                               ctypes.byref(h)) == abi.PERF_ENOMEM
    cams[3].fx = float("nan")
    assert lib.perf_init_scene(ctypes.byref(d), cams, 8, None, ctypes.c_void_p(4096), n, None,
                               ctypes.byref(h)) == abi.PERF_EINVAL
    assert "camera 3" in lib.perf_last_error().decode()
    assert lib.perf_init_scene(ctypes.byref(d), cams, 8, None, ctypes.c_void_p(4096), n, None, None) == abi.PERF_EINVAL
    assert lib.perf_gn_step(None, None, None, None) == abi.PERF_EINVAL
    assert lib.perf_pack_bf16(None, None, -1, None) == abi.PERF_EINVAL


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2112_05598_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "perf_oracle" not in text, fn


def test_upsample_rejects_mismatched_levels():
    """perf_upsample validates the two descriptors before any device work."""
    import ctypes
    import perf_synth as ps
    from paper_2112_05598_amd import abi
    from paper_2112_05598_amd.scene import make_desc
    lib = abi.load()
    a = ps.SceneSpec(8, 8, 8, layer_radii=(1.8,), env_w=16, env_h=8)
    fake = ctypes.c_void_p(256)  # never dereferenced: every case below fails validation first
    cases = [
        (a, ps.SceneSpec(16, 16, 16, bbox_min=(-1, -1, -2), layer_radii=(1.8,), env_w=32, env_h=16)),  # box
        (a, ps.SceneSpec(16, 16, 16, layer_radii=(1.8, 3.0), env_w=32, env_h=16)),                     # layers
        (a, ps.SceneSpec(16, 16, 16, layer_radii=(2.0,), env_w=32, env_h=16)),                         # radii
        (a, ps.SceneSpec(1, 16, 16, layer_radii=(1.8,), env_w=32, env_h=16)),                          # dims
    ]
    for sf, st in cases:
        rc = lib.perf_upsample(ctypes.byref(make_desc(sf, 1, 1)), fake, ctypes.byref(make_desc(st, 1, 1)), fake, None)
        assert rc == abi.PERF_EINVAL, (sf, st, rc)
    rc = lib.perf_upsample(ctypes.byref(make_desc(a, 1, 1)), None, ctypes.byref(make_desc(a, 1, 1)), fake, None)
    assert rc == abi.PERF_EINVAL


def test_invert_blocks_rejects_bad_arguments_before_device_work():
    """perf_invert_blocks validates its arguments before any launch; zero units is a no-op."""
    import ctypes
    from paper_2112_05598_amd import abi
    lib = abi.load()
    fake = ctypes.c_void_p(256)  # never dereferenced: every case below returns before a launch
    assert lib.perf_invert_blocks(None, 4, abi.PERF_PRECOND_JACOBI, fake, None) == abi.PERF_EINVAL
    assert lib.perf_invert_blocks(fake, 4, abi.PERF_PRECOND_BLOCK4, None, None) == abi.PERF_EINVAL
    assert lib.perf_invert_blocks(fake, -1, abi.PERF_PRECOND_JACOBI, fake, None) == abi.PERF_EINVAL
    for kind in (abi.PERF_PRECOND_NONE, abi.PERF_PRECOND_LEARNED, 17):
        assert lib.perf_invert_blocks(fake, 4, kind, fake, None) == abi.PERF_EINVAL
    assert lib.perf_invert_blocks(None, 0, abi.PERF_PRECOND_JACOBI, None, None) == abi.PERF_OK
