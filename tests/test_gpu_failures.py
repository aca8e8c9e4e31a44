"""Failure handling, forced from the host (no kernel is made to fault): a coarse
propagator that is much worse than the fine one must shorten the adaptive windows exactly
as the oracle's literal driver does; a non-finite state inside a corrected iteration must
be reported with the slab (and system) it appeared in; more neighbours than the lists
hold must be reported as an overflow."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import parareal as OPR
from paper_2212_10508_amd import workloads as W

pytestmark = pytest.mark.gpu

QTOL = 1e-8


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_10508_amd import snapmd
    return snapmd


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


FS10 = {k: (v * 10.0 if k in ("A", "c0", "c1", "c2") else v) for k, v in W.FS_W.items()}


@pytest.mark.parametrize("coarse_fs", [None, FS10], ids=["fs", "fs_x10"])
def test_bad_coarse_potential_shortens_windows_like_oracle(S, coarse_fs):
    """Coarse forces ten times the fine potential's Finnis-Sinclair part (every energy
    coefficient x10): the iterates disagree more, the relative error passes the explosion
    threshold and the windows shorten; the GPU takes the same decisions as the oracle."""
    from paper_2212_10508_amd import parareal as PR
    J, N, L = 2, 6, 10
    x, box = W.bcc_sia(4, jitter=0.05, seed=21)
    p = W.maxwell_momenta(x.shape[1], 1000.0, seed=21)
    beta = W.snap_beta(J, seed=21, scale=2e-2)
    snap = dict(J=J, beta=beta, rcut=W.SNAP_RCUT, rfac0=W.SNAP_RFAC0, rmin0=0.0)
    prop = OPR.Propagators(box=box, L=L, dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=5, noise_id=2,
                           snap=snap, fs=W.FS_W, coarse_fs=coarse_fs)
    olog = []
    tref, nad_ref, kc_ref = OPR.parareal_adaptive(prop, x, p, N, 1e-10, 1e-2, log=olog)
    ctx = S.Context(0)
    ctx.set_coarse_fs(coarse_fs)
    log = []
    q, _, nad, kc = PR.adaptive_parareal(ctx, dev(x), dev(p), box, N, L, 1e-10, 1e-2, dt=1e-3, gamma=1.0,
                                         mass=W.MASS_W, T=1000.0, seed=5, noise_id=2, fs=W.FS_W, J=J, beta=beta,
                                         log=log)
    print("coarse %s: windows %s" % ("x10" if coarse_fs else "fs", [(a["n_in"], a["n_fi"], a["n_fi_after"])
                                                                 for a in log]), flush=True)
    assert (nad, kc) == (nad_ref, kc_ref)
    assert [(a["n_in"], a["n_fi"], a["n_fi_after"]) for a in log] == \
           [(a["n_in"], a["n_fi"], a["n_fi_after"]) for a in olog]
    qh = q.cpu().numpy()
    for n in range(N + 1):
        assert np.abs(qh[n] - tref[n][0]).max() < QTOL
    if coarse_fs is None:
        assert nad == 1
    else:
        assert nad > 1 and any(a["n_fi_after"] < a["n_fi"] for a in log)


def test_nonfinite_in_corrected_iteration_names_the_slab(S):
    """A NaN planted (from the host) in the slab-3 start state between the window
    initialisation and the corrected iteration: the jump J_3 is not finite, the sweep
    stops there and the call reports slab 3."""
    J, N, L = 2, 5, 3
    x, box = W.bcc_sia(4, jitter=0.05, seed=22)
    p = W.maxwell_momenta(x.shape[1], 1000.0, seed=22)
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=4, noise_id=0, fs=W.FS_W)
    ctx = S.Context(0)
    n = x.shape[1]
    q = torch.zeros((N + 1, 3, n), dtype=torch.float64, device="cuda")
    pq, qp, pp = torch.zeros_like(q), torch.zeros_like(q), torch.zeros_like(q)
    q[0], pq[0] = dev(x), dev(p)
    ctx.parareal_iterate(None, None, q, pq, box, L, 0, N, 1e100, **kw)
    pq[3, 1, 7] = float("nan")
    with pytest.raises(S.SnapmdError) as e:
        ctx.parareal_iterate(qp, pp, q, pq, box, L, 0, N, 1e100, J=J, beta=W.snap_beta(J, seed=22), **kw)
    assert e.value.code == S.ENONFINITE and "slab 3" in str(e.value)
    # slabs before the bad one were corrected and are finite
    assert torch.isfinite(q[:4]).all()


def test_nonfinite_in_pipelined_iterations_matches_synchronous(S):
    """The same planted NaN with two corrected iterations enqueued back to back
    (parareal_iterate_async): each collect reports what the synchronous calls report, in
    order (slab 3, then slab 4: the second iteration starts from the first one's states,
    whose slab-4 start is the non-finite value the first sweep stopped at), and the
    states end equal bitwise."""
    J, N, L = 2, 5, 3
    x, box = W.bcc_sia(4, jitter=0.05, seed=22)
    p = W.maxwell_momenta(x.shape[1], 1000.0, seed=22)
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=4, noise_id=0, fs=W.FS_W)
    beta = W.snap_beta(J, seed=22)
    ctx = S.Context(0)
    n = x.shape[1]
    out = []
    for pipelined in (False, True):
        q = torch.zeros((N + 1, 3, n), dtype=torch.float64, device="cuda")
        pq, qp, pp = torch.zeros_like(q), torch.zeros_like(q), torch.zeros_like(q)
        q[0], pq[0] = dev(x), dev(p)
        ctx.parareal_iterate(None, None, q, pq, box, L, 0, N, 1e100, **kw)
        pq[3, 1, 7] = float("nan")
        errs = []
        if pipelined:
            for _ in range(2):
                ctx.parareal_iterate_async(qp, pp, q, pq, box, L, 0, N, 1e100, J=J, beta=beta, **kw)
            for _ in range(2):
                with pytest.raises(S.SnapmdError) as e:
                    ctx.parareal_collect()
                errs.append((e.value.code, str(e.value)))
        else:
            for _ in range(2):
                with pytest.raises(S.SnapmdError) as e:
                    ctx.parareal_iterate(qp, pp, q, pq, box, L, 0, N, 1e100, J=J, beta=beta, **kw)
                errs.append((e.value.code, str(e.value)))
        torch.cuda.synchronize()
        out.append((errs, [t.cpu().numpy() for t in (q, pq, qp, pp)]))
    (e0, s0), (e1, s1) = out
    assert [c for c, _ in e0] == [S.ENONFINITE] * 2 and "slab 3" in e0[0][1] and "slab 4" in e0[1][1]
    assert e1 == e0
    for a, b in zip(s0, s1):
        assert np.array_equal(a, b, equal_nan=True)


def test_nonfinite_in_batch_names_system_and_slab(S):
    J, N, L = 2, 4, 3
    xs, ps, boxes = [], [], []
    for k in range(2):
        x, box = W.bcc_sia(4, jitter=0.05, seed=23 + k)
        xs.append(x)
        ps.append(W.maxwell_momenta(x.shape[1], 1000.0, seed=23 + k))
        boxes.append(box)
    off = np.array([0, xs[0].shape[1], xs[0].shape[1] + xs[1].shape[1]], dtype=np.int32)
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=[1000.0, 900.0], seed=4, noise_id=[0, 1], fs=W.FS_W)
    ctx = S.Context(0)
    q = torch.zeros((N + 1, 3, int(off[-1])), dtype=torch.float64, device="cuda")
    pq, qp, pp = torch.zeros_like(q), torch.zeros_like(q), torch.zeros_like(q)
    q[0] = dev(np.concatenate(xs, axis=1))
    pq[0] = dev(np.concatenate(ps, axis=1))
    ctx.parareal_iterate_batch(None, None, q, pq, off, boxes, L, [0, 0], [N, N], 1e100, **kw)
    pq[2, 0, int(off[1]) + 11] = float("nan")      # system 1, slab 2
    with pytest.raises(S.SnapmdError) as e:
        ctx.parareal_iterate_batch(qp, pp, q, pq, off, boxes, L, [0, 0], [N, N], 1e100, J=J,
                                   beta=W.snap_beta(J, seed=23), **kw)
    assert e.value.code == S.ENONFINITE and "system 1" in str(e.value) and "slab 2" in str(e.value)


def _compressed():
    # bcc at a = 2.2 A: about 100 atoms within the 5.03 A list radius of SNAP (64 fit)
    x, box = W.bcc_sia(6, a=2.2, jitter=0.0, interstitial=False)
    return x, box


def test_neighbour_overflow_is_reported(S):
    x, box = _compressed()
    n = x.shape[1]
    ctx = S.Context(0)
    beta = W.snap_beta(2, seed=1)
    ctx.snap_forces(dev(x), [0, n], box, 2, beta)
    with pytest.raises(S.SnapmdError) as e:
        ctx.sync()
    assert e.value.code == S.EOVERFLOW
    # the error is cleared: a normal system works afterwards
    x2, box2 = W.bcc_sia(4, jitter=0.05, seed=1)
    f = ctx.snap_forces(dev(x2), [0, x2.shape[1]], box2, 2, beta)
    ctx.sync()
    assert torch.isfinite(f).all()


def test_coarse_sweep_overflow_is_reported(S):
    """The coarse sweep's own list (48 entries per atom) overflows on the compressed
    lattice; one slab of one step."""
    x, box = _compressed()
    n = x.shape[1]
    ctx = S.Context(0)
    q = torch.zeros((2, 3, n), dtype=torch.float64, device="cuda")
    pq = torch.zeros_like(q)
    q[0] = dev(x)
    with pytest.raises(S.SnapmdError) as e:
        ctx.parareal_iterate(None, None, q, pq, box, 1, 0, 1, 1e100, dt=1e-3, gamma=1.0, mass=W.MASS_W, T=0.0,
                             seed=1, noise_id=0, fs=W.FS_W)
    assert e.value.code == S.EOVERFLOW
