"""CPU-only checks of the HIP library: it loads, exports every symbol the header declares, and the
input generators have the shapes the workloads state.  No compute call is made (no GPU here)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2502_10872_amd import inputs as I
from paper_2502_10872_amd import shell as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "shell.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(shell_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def library():
    if not os.path.exists(S.LIBRARY):
        pytest.skip("libshell_hip.so not built (run __graft_entry__.build())")
    return S.lib()


def test_library_exports_every_header_symbol(library):
    syms = header_symbols()
    assert len(syms) >= 15
    for name in syms:
        assert hasattr(library, name), name
    assert set(S.EXPORTS) == set(syms)


def test_library_has_gfx950_code_object(library):
    data = open(S.LIBRARY, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_status_strings_need_no_device(library):
    assert S.shell_status_string(0) == "ok"
    assert S.shell_status_string(4) == "degenerate stencil"


def test_struct_layouts_match_header():
    assert ctypes.sizeof(S.shell_material_t) == 32
    assert ctypes.sizeof(S.shell_config_t) == 16 and S.shell_config_t.flags.offset == 12
    assert ctypes.sizeof(S.shell_step_stats_t) == 4 * 4 + 2 * 8 + 256 * 3 * 4
    assert ctypes.sizeof(S.shell_step_params_t) == 8 + 24 + 8 + 16 + 8 + 8 + 8
    assert ctypes.sizeof(S.shell_static_params_t) == 8 + 8 + 8 + 8 + 8 + 16 + 8
    assert S.shell_static_params_t.pcg_rtol.offset == 32 and S.shell_static_params_t.replay_counts.offset == 56
    assert ctypes.sizeof(S.shell_profile_t) == S.SHELL_NUM_PHASES * (8 + 8)
    assert ctypes.sizeof(S.shell_hessian_info_t) == 5 * 8 + 2 * 4


def test_batch_step_refuses_a_stats_count_other_than_the_member_count():
    # the stats buffer holds one record per member: a wrong count is refused before the library is called
    params, _keep = S.step_params(1 / 60)
    fake = 0x7E57
    S._batch_members[fake] = 3
    try:
        with pytest.raises(ValueError, match="3 members"):
            S.shell_batch_step(fake, params, 1)
    finally:
        S._batch_members.pop(fake, None)


def test_workload_shapes():
    m = I.workload_plate32()
    assert m.nv == 1024 and m.nt == 1922 and m.pinned.sum() == 64
    c = I.workload_cylinder(64)
    assert c.nv == 4096 and c.nt == 2 * 63 * 63
    assert np.allclose(np.linalg.norm(c.X[:, [0]] * 0 + (c.X[:, [0, 2]] + [0, 0.5]), axis=1), 0.5)
    R = I.sphere_cap_radius()
    assert 0.3 <= R <= 2.0
    cap = I.sphere_cap_mesh(16, R, 1.2 * R, 0.2, 3)
    assert np.allclose(np.linalg.norm(cap.X + [0, 0, R], axis=1), R)


def test_jitter_is_seeded_and_interior_only():
    a = I.plate_mesh(12, 1.0, 0.2, 5)
    b = I.plate_mesh(12, 1.0, 0.2, 5)
    c = I.plate_mesh(12, 1.0, 0.0, 5)
    assert np.array_equal(a.X, b.X)
    ring = I.grid_boundary_mask(12, 12)
    assert np.array_equal(a.X[ring], c.X[ring])
    d = np.abs(a.X - c.X)[~ring]
    assert d.max() < 0.2 / 11 and d.max() > 0.1 / 11


def test_batch_and_serving_generators():
    specs = I.batch_specs()
    assert len(specs) == 64
    assert all(16 <= s["n"] <= 512 for s in specs)
    assert [s["model"] for s in specs[:6]] == list(I.MODELS)
    tr = I.serving_trace(rate=200.0, duration=5.0)
    assert 800 < len(tr) < 1200
    nv = np.array([r["n"] ** 2 for r in tr])
    assert nv.min() >= 1600 and nv.max() <= 1_000_000 + 2000
