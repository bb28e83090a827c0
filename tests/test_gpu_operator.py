"""GPU parity of the aperture operator A = D(a) F, A^H and A^H A (Sec. II-B,
eq. A) against the float64 oracle, through the C ABI."""

import numpy as np
import pytest

import oracle
from helpers import rel_l2, report

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def C():
    import torch  # noqa: F401
    import paper_2406_13651_amd._clamp as C
    return C


def _run(C, scene, direction, x, nbatch):
    import torch
    plan = C.clamp_plan_create([scene])
    ws = plan.workspace()
    xt = torch.from_numpy(x.astype(np.complex64)).cuda()
    out = torch.empty_like(xt)
    C.clamp_aperture_op(plan, 0, direction, xt, out, nbatch, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy(), plan


CASES = [
    # nx, ny, nz, looks, radius, nbatch
    (32, 32, 16, 4, 8.0, 4),       # the tiny workload's geometry
    (256, 256, 3, 2, 64.0, 3),     # 129 band columns: 9 tiles with a ragged last tile, chunked batch
    (128, 64, 2, 2, 20.0, 2),      # nx != ny
    (192, 192, 2, 1, 48.0, 1),     # radix-3 length
    (384, 128, 1, 1, 40.0, 2),     # radix-3 rows, chunked batch of 1 look
    (512, 512, 1, 1, 128.0, 1),    # largest length
    (64, 64, 5, 3, 31.0, 3),       # pupil almost filling the grid
]


@pytest.mark.parametrize("nx,ny,nz,looks,radius,nbatch", CASES)
def test_operator_matches_oracle(C, nx, ny, nz, looks, radius, nbatch):
    rng = np.random.default_rng(nx * 7 + ny * 3 + nz)
    scene = C.Scene(nx, ny, nz, looks, radius)
    shape = (nbatch, nz, ny, nx)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    mask = oracle.pupil_mask(ny, nx, radius)
    x64 = x.astype(np.complex128)
    for direction, ref in ((C.CLAMP_FWD, oracle.apply_A(x64, mask)),
                           (C.CLAMP_ADJ, oracle.apply_AH(x64, mask)),
                           (C.CLAMP_NORMAL, oracle.apply_AHA(x64, mask))):
        got, plan = _run(C, scene, direction, x, nbatch)
        err = report("aperture dir=%d %dx%dx%d R=%g" % (direction, nx, ny, nz, radius), rel_l2(got, ref), TOL)
        assert err <= TOL
        if direction == C.CLAMP_FWD:
            assert np.all(got[:, :, ~mask] == 0)


def test_all_pass_mask_is_identity(C):
    rng = np.random.default_rng(5)
    nx = ny = 64
    scene = C.Scene(nx, ny, 2, 2, mask=np.ones((ny, nx), dtype=np.uint8))
    x = (rng.standard_normal((2, 2, ny, nx)) + 1j * rng.standard_normal((2, 2, ny, nx))).astype(np.complex64)
    got, plan = _run(C, scene, C.CLAMP_NORMAL, x, 2)
    assert plan.info[0]["P"] == nx * ny and plan.info[0]["alpha"] == 1.0
    assert report("all-pass A^H A = I", rel_l2(got, x), TOL) <= TOL


def test_adjoint_and_parseval_on_gpu(C):
    import torch
    rng = np.random.default_rng(11)
    nx = ny = 256
    nz = 4
    scene = C.Scene(nx, ny, nz, 1, 64.0)
    plan = C.clamp_plan_create([scene])
    ws = plan.workspace()
    x = (rng.standard_normal((1, nz, ny, nx)) + 1j * rng.standard_normal((1, nz, ny, nx))).astype(np.complex64)
    y = (rng.standard_normal((1, nz, ny, nx)) + 1j * rng.standard_normal((1, nz, ny, nx))).astype(np.complex64)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    ax, ahy = torch.empty_like(xt), torch.empty_like(yt)
    C.clamp_aperture_op(plan, 0, C.CLAMP_FWD, xt, ax, 1, ws)
    C.clamp_aperture_op(plan, 0, C.CLAMP_ADJ, yt, ahy, 1, ws)
    ax, ahy = ax.cpu().numpy().astype(np.complex128), ahy.cpu().numpy().astype(np.complex128)
    lhs = np.vdot(ax, y.astype(np.complex128))
    rhs = np.vdot(x.astype(np.complex128), ahy)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    # A A^H = D(a): the forward map of A^H y is y on the pupil, and ||A^H y|| = ||D(a) y||
    mask = oracle.pupil_mask(ny, nx, 64.0)
    assert np.isclose(np.linalg.norm(ahy), np.linalg.norm(y[:, :, mask]), rtol=1e-5)
    # projector: ||A^H A x|| <= ||x||
    assert np.linalg.norm(ax) <= np.linalg.norm(x)


def test_pupil_index_is_column_major_disk(C):
    scene = C.Scene(256, 256, 1, 1, 64.0)
    plan = C.clamp_plan_create([scene])
    idx = C.clamp_plan_pupil_index(plan, 0)
    mask = oracle.pupil_mask(256, 256, 64.0)
    assert plan.info[0]["P"] == mask.sum() == 12853
    assert np.isclose(plan.info[0]["alpha"], oracle.aperture_fraction(mask))
    u, v = idx // 256, idx % 256
    assert np.all(mask[u, v])
    key = v.astype(np.int64) * 256 + u
    assert np.all(np.diff(key) > 0)  # column by column, rows increasing


def test_zero_batch_and_errors(C):
    import torch
    scene = C.Scene(64, 64, 2, 2, 16.0)
    plan = C.clamp_plan_create([scene])
    ws = plan.workspace()
    x = torch.zeros(2, 2, 64, 64, dtype=torch.complex64, device="cuda")
    C.clamp_aperture_op(plan, 0, C.CLAMP_FWD, x, x.clone(), 0, ws)
    with pytest.raises(C.ClampError):
        C.clamp_aperture_op(plan, 0, 7, x, x.clone(), 1, ws)
    with pytest.raises(C.ClampError):
        C.clamp_aperture_op(plan, 0, C.CLAMP_FWD, x, x, 1, ws)  # in and out overlap


def test_prior_rejects_misaligned_input(C):
    """The prior's x pass reads its input in float4 units: a pointer that is
    not 16-byte aligned is an argument error, not a fault."""
    import torch
    scene = C.Scene(64, 32, 4, 2, 8.0)
    plan = C.clamp_plan_create([scene])
    ws = plan.workspace()
    n = 64 * 32 * 4
    buf = torch.zeros(n + 4, dtype=torch.float32, device="cuda")
    out = torch.zeros(n, dtype=torch.float32, device="cuda")
    C.clamp_prior_gauss(plan, 0, 1.0, buf[4:], out, ws)  # 16-byte offset: accepted
    with pytest.raises(C.ClampError, match="aligned"):
        C.clamp_prior_gauss(plan, 0, 1.0, buf[1:n + 1], out, ws)
    torch.cuda.synchronize()
