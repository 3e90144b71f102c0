"""The transforms Q of Sec. 5 built on the GPU (identity, DCT; U3 has its own
tests) against the float64 oracle, the Stiefel check on many column pairs,
the CholeskyQR2 re-orthonormalisation of Q, and Thms. 4.3 and 4.6 on the
GPU's own results."""

import numpy as np
import pytest

import oracle
from helpers import dev, devq, host, rel, say
from paper_2409_19402_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2409_19402_amd import binding
    return binding


@pytest.mark.parametrize("n3,p", [(2, 2), (16, 4), (200, 20), (224, 32), (257, 257)])
def test_build_q(pq, n3, p):
    import torch
    say(f"build_q n3={n3} p={p}")
    # float64: the oracle rounds the angle pi (2t + 1) l / (2 n3) (up to about
    # pi n3) before the cosine, an absolute error near n3 * 2^-52 that the
    # kernel's exact reduction of (2t + 1) l mod 4 n3 does not have
    for dt, tol in ((torch.float32, 1e-6), (torch.float64, max(1e-14, 4e-16 * n3))):
        Qd = pq.build_q("dct", n3, p, dt)
        assert np.max(np.abs(host(Qd) - oracle.dct_q(n3, p))) <= tol
        Qi = pq.build_q("identity", n3, p, dt)
        np.testing.assert_array_equal(host(Qi), oracle.identity_q(n3, p))
        assert pq.check_q(Qd).item() <= (1e-6 if dt == torch.float32 else 1e-13)


def test_build_q_rejects(pq):
    from paper_2409_19402_amd._lib import ProjProdError
    with pytest.raises(ValueError):
        pq.build_q("random", 8, 2)
    with pytest.raises(ProjProdError):
        pq.build_q("dct", 4, 5)  # p > n3


def test_check_q_many_pairs(pq):
    """p = 64: 2080 column pairs over many workgroups; one perturbed entry
    fixes the maximum."""
    rng = np.random.default_rng(8)
    Q = synth.random_orthonormal(rng, 300, 64)
    assert pq.check_q(devq(Q)).item() == pytest.approx(oracle.check_q(Q), abs=1e-15)
    Qp = Q.copy()
    Qp[17, 40] += 1e-3
    assert pq.check_q(devq(Qp)).item() == pytest.approx(oracle.check_q(Qp), rel=1e-12)


def test_check_q_flag(pq):
    """The device-side flag of the Def. 3.1 precondition: 0 for orthonormal Q
    (float32 and float64), 1 once one entry is perturbed beyond the tolerance
    and for a NaN entry; the distance matches the oracle's."""
    import torch
    rng = np.random.default_rng(9)
    Q = synth.random_orthonormal(rng, 300, 64)
    for dt, tol in ((torch.float32, 1e-6), (torch.float64, 1e-13)):
        Qd = devq(Q.astype(np.float32 if dt == torch.float32 else np.float64))
        dist, flag = pq.check_q_flag(Qd, tol)
        assert flag.item() == 0
        assert dist.item() == pytest.approx(pq.check_q(Qd).item(), abs=0)
    Qp = Q.copy()
    Qp[17, 40] += 1e-3
    dist, flag = pq.check_q_flag(devq(Qp), 1e-5)
    assert flag.item() == 1
    assert dist.item() == pytest.approx(oracle.check_q(Qp), rel=1e-12)
    _, flag = pq.check_q_flag(devq(Qp), 1.0)  # within a loose tolerance
    assert flag.item() == 0
    Qn = Q.copy()
    Qn[3, 5] = np.nan
    dist, flag = pq.check_q_flag(devq(Qn), 1.0)
    assert flag.item() == 1 and np.isnan(dist.item())


def test_info_entries_all_written(pq):
    """The info arrays come back from torch.empty: the library writes every
    entry of them (checked here on arrays filled with a sentinel first)."""
    import torch
    c = synth.tiny()
    A = dev(c["A"].astype(np.float32))
    Q = devq(c["Q"].astype(np.float32))
    k = c["k"]
    sentinel = -12345
    for n, call in ((3, lambda i: pq.tsvdq(A, Q, k, info=i)),
                    (3, lambda i: pq.svdii(A, Q, 0.9, info=i)),
                    (3, lambda i: pq.u3(A, 4, info=i)),
                    (4, lambda i: pq.tsvdq_backward(A, Q, k, sbar=torch.ones(k, Q.shape[1], device="cuda"),
                                                    info=i))):
        info = torch.full((n,), sentinel, dtype=torch.int32, device="cuda")
        call(info)
        got = info.cpu().tolist()
        assert all(v >= 0 for v in got), got
    info = torch.full((1,), sentinel, dtype=torch.int32, device="cuda")
    qs = torch.empty_like(Q)
    import paper_2409_19402_amd._lib as L
    ws = torch.empty(L.load().pq_orthonormalize_q_workspace(*Q.shape), dtype=torch.uint8, device="cuda")
    L.call("pq_orthonormalize_q", Q.data_ptr(), 0, Q.shape[0], Q.shape[1], qs.data_ptr(), info.data_ptr(),
           ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    assert info.item() == 0


def test_thm_4_3_and_4_6_on_gpu_results(pq):
    """Video-shaped data: the projection error with Q = U3 (GPU) is no larger
    than with the DCT or the identity (Thm. 4.3), and the GPU tSVDQ with
    Q = U3 and k = min(k1, k2) is no worse than the truncated HOSVD of
    multilinear rank (k1, k2, p) (Thm. 4.6)."""
    rng = np.random.default_rng(33)
    A_st = synth.video(rng, 40, 56, 48)
    Al = synth.logical(A_st)
    A = dev(A_st)
    n3, p = 48, 8
    QU, _, info = pq.u3(A, p)
    assert int(info[1].item()) == 0
    errs = {}
    for name, Q in (("u3", QU), ("dct", pq.build_q("dct", n3, p)), ("identity", pq.build_q("identity", n3, p))):
        errs[name] = oracle.fro2(Al - host(pq.proj(A, Q)))
    say(f"projection errors {errs}")
    assert errs["u3"] <= errs["dct"] * (1 + 1e-6) and errs["u3"] <= errs["identity"] * (1 + 1e-6)
    for k1, k2 in ((6, 9), (12, 4)):
        k = min(k1, k2)
        t = pq.tsvdq(A, QU, k, approx=True)
        e_t = oracle.fro2(Al - host(t.Ak))
        e_h = oracle.fro2(Al - oracle.hosvd(Al, k1, k2, p))
        say(f"Thm 4.6 k1={k1} k2={k2}: tSVDQ {e_t:.6e} <= HOSVD {e_h:.6e}")
        assert e_t <= e_h * (1 + 1e-6)


@pytest.mark.parametrize("n3,p", [(16, 4), (200, 20), (257, 33), (130, 128), (5, 1), (64, 64)])
def test_orthonormalize_q(pq, n3, p):
    """Q pushed off the Stiefel manifold, re-orthonormalised on the GPU,
    against the oracle on the values the GPU sees (float32 input widened)."""
    import torch
    say(f"orthonormalize_q n3={n3} p={p}")
    rng = np.random.default_rng(70 + p)
    Qp = synth.random_orthonormal(rng, n3, p) + 1e-3 * rng.standard_normal((n3, p))
    for dt, tol, otol in ((np.float64, 1e-13, 1e-14), (np.float32, 1.5e-7, 2e-6)):
        Qin = devq(Qp.astype(dt))
        out, info = pq.orthonormalize_q(Qin)
        assert int(info.item()) == 0
        ref, rinfo = oracle.orthonormalize_q(host(Qin))
        assert rinfo == 0
        assert np.max(np.abs(host(out) - ref)) <= tol
        assert pq.check_q(out).item() <= otol
        # in place
        pq.orthonormalize_q(Qin, out=Qin)
        assert torch.equal(Qin, out)


def test_orthonormalize_q_dependent_column_and_rejects(pq):
    import torch
    from paper_2409_19402_amd._lib import ProjProdError
    rng = np.random.default_rng(71)
    Q = synth.random_orthonormal(rng, 30, 5)
    Q[:, 3] = Q[:, 0] + 0.5 * Q[:, 1]
    Qd = devq(Q)
    sentinel = torch.full_like(Qd, 7.0)
    _, info = pq.orthonormalize_q(Qd, out=sentinel)
    assert int(info.item()) == 4
    assert bool((sentinel == 7.0).all())  # left unwritten
    with pytest.raises(ProjProdError):
        pq.orthonormalize_q(devq(synth.random_orthonormal(rng, 300, 129)))  # p > 128
