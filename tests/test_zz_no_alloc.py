"""The allocation-free SNAP forces (snap_forces_noalloc) against snap_forces, through
the C ABI: two calls in a row, the second on a smaller batch, must give the same forces
and energies (bitwise in the kernel shape the allocation-free path runs, to rounding in
the built-in one); sizes beyond the scratch limits are refused before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2212_10508_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_10508_amd import snapmd
    return snapmd


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _batch(ncells, seed):
    xs, boxes = [], []
    for k, n in enumerate(ncells):
        x, box = W.bcc_sia(n, jitter=0.1, seed=seed + k)
        xs.append(x)
        boxes.append(box)
    off = np.concatenate([[0], np.cumsum([x.shape[1] for x in xs])]).astype(np.int32)
    return np.concatenate(xs, axis=1), off, np.array(boxes)


@pytest.mark.parametrize("J", [6, 8])
def test_noalloc_matches_snap_forces_on_two_calls(S, J):
    beta = W.snap_beta(J, seed=J, scale=1e-2)
    ctx = S.Context(0)
    # a 1025 + 433 + 129 atom batch (1587 atoms), then a single 129-atom system
    for ncells, seed in (((8, 6, 4), 3), ((4,), 9)):
        x, off, boxes = _batch(ncells, seed)
        N = x.shape[1]
        print("noalloc J=%d: %d systems, %d atoms" % (J, len(off) - 1, N), flush=True)
        xd = dev(x)
        f_ref = torch.empty((3, N), dtype=torch.float64, device="cuda")
        e_ref = torch.empty(N, dtype=torch.float64, device="cuda")
        ctx.set_kernel_shape(J, None)  # built-in shape: the density split of small launches
        f_def = ctx.snap_forces(xd, off, boxes, J, beta).clone()
        ctx.set_kernel_shape(J, (45, 0, 12, 1))  # the shape the allocation-free path runs
        ctx.snap_forces(xd, off, boxes, J, beta, f=f_ref, e_atom=e_ref)
        ctx.set_kernel_shape(J, None)
        f = torch.full((3, N), float("nan"), dtype=torch.float64, device="cuda")
        e = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.snap_forces_noalloc(xd, off, boxes, J, beta, f, e_atom=e)
        ctx.sync()
        fmax = torch.max(torch.abs(f_ref)).item()
        assert torch.max(torch.abs(f - f_ref)).item() <= 1e-12 * fmax
        assert torch.max(torch.abs(e - e_ref)).item() <= 1e-12 * torch.max(torch.abs(e_ref)).item()
        assert torch.equal(f, f_ref) and torch.equal(e, e_ref)   # same kernels, same order
        assert torch.max(torch.abs(f - f_def)).item() <= 1e-12 * fmax
        # accumulate mode adds onto f
        ctx.snap_forces_noalloc(xd, off, boxes, J, beta, f, accumulate=True)
        ctx.sync()
        assert torch.max(torch.abs(f - 2 * f_ref)).item() <= 1e-12 * fmax


def test_noalloc_refuses_sizes_beyond_its_limits(S):
    ctx = S.Context(0)
    J = 2
    beta = W.snap_beta(J, seed=1)
    x, box = W.bcc_sia(10, seed=1)      # 2001 atoms fit
    x2 = np.concatenate([x, x[:, :48]], axis=1)   # 2049 atoms do not
    f = torch.empty((3, x2.shape[1]), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SnapmdError) as e:
        ctx.snap_forces_noalloc(dev(x2), [0, x2.shape[1]], box, J, beta, f)
    assert e.value.code == S.EINVAL and "at most 2048 atoms" in str(e.value)
    offs = np.arange(258, dtype=np.int32)   # 257 one-atom systems
    with pytest.raises(S.SnapmdError) as e:
        ctx.snap_forces_noalloc(dev(x[:, :257]), offs, np.tile(box, (257, 1)), J, beta, f[:, :257].contiguous())
    assert e.value.code == S.EINVAL and "n_sys" in str(e.value)
