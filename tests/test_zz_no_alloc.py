"""The no-allocation force entry point (shell_eval_forces_noalloc) against shell_eval_forces, through the
C ABI: two calls in a row on one device, the second on a smaller mesh, both precisions, with and without
the membrane."""

import numpy as np
import pytest

from paper_2502_10872_amd import inputs as I
from paper_2502_10872_amd import shell as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAT = I.MATERIAL


def forces(fn, st, x, f32):
    xd = torch.tensor(x, device="cuda:0")
    fd = torch.full(x.shape, float("nan"), dtype=torch.float32 if f32 else torch.float64, device="cuda:0")
    ed = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
    fn(st, xd, fd, ed)
    torch.cuda.synchronize()
    return fd.double().cpu().numpy(), ed.item()


@pytest.mark.parametrize("precision", [S.SHELL_PREC_FP64, S.SHELL_PREC_MIXED])
@pytest.mark.parametrize("flags", [0, S.SHELL_FLAG_MEMBRANE])
def test_noalloc_forces_equal_the_allocating_entry_point(precision, flags):
    """Same kernels, same inputs: the forces and energy agree to the bit (every sum has a fixed order),
    for a 256 x 256 cap and then a smaller 64 x 64 cylinder reusing the same scratch."""
    f32 = precision == S.SHELL_PREC_MIXED
    for mesh, model in ((I.workload_sphere_cap(256, "SS"), "SS"), (I.workload_cylinder(64, "FS"), "FS")):
        x = mesh.X + 1e-3 * I.rng(5).standard_normal(mesh.X.shape)
        st = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, precision=precision, flags=flags)
        try:
            fa, ea = forces(S.shell_eval_forces, st, x, f32)
            fb, eb = forces(S.shell_eval_forces_noalloc, st, x, f32)
        finally:
            S.shell_destroy_stencils(st)
        assert np.isfinite(fa).all() and np.array_equal(fa, fb)
        assert ea == eb


def test_noalloc_rejects_meshes_beyond_its_scratch():
    mesh = I.plate_mesh(1200, 1.0, 0.0, 0, "EP", "none")  # 1.44M vertices: more than the 64 MiB holds
    st = S.shell_build_stencils(mesh.X, mesh.tris, "EP", MAT)
    try:
        x = torch.tensor(mesh.X, device="cuda:0")
        f = torch.zeros_like(x)
        with pytest.raises(S.ShellError) as ei:
            S.shell_eval_forces_noalloc(st, x, f)
        assert ei.value.status == S.SHELL_E_INVALID_ARG
    finally:
        S.shell_destroy_stencils(st)
