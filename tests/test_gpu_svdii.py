"""*_Q-SVDII (Alg. 4.2) on the GPU against the float64 oracle: the multirank
rho from the global energy threshold is compared exactly (gamma is placed
halfway between two consecutive cumulative energies of the oracle, so that
rounding cannot move K), the kept singular values and the approximation
elementwise, and Thms. 4.4 and 4.5 on the GPU's own results."""

import numpy as np
import pytest

import oracle
from helpers import relmax, dev, devq, host, rel, say
from paper_2409_19402_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-10


@pytest.fixture(scope="module")
def pq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2409_19402_amd import binding
    return binding


def _gamma_between(s_all, K):
    """An energy level strictly between the cumulative energies of the first
    K - 1 and the first K values of the global descending order, so that
    Alg. 4.2 selects exactly K of them."""
    v = np.sort(s_all.ravel())[::-1] ** 2
    e = np.cumsum(v) / v.sum()
    lo = e[K - 2] if K >= 2 else 0.0
    return 0.5 * (lo + e[K - 1])


def _case(seed, n1, n2, n3, p, dtype):
    rng = np.random.default_rng(seed)
    A = synth.gaussian(rng, n1, n2, n3, dtype)
    Q = synth.random_orthonormal(rng, n3, p)
    return A, Q


def _check_factors(out, ref_s_all, rho, kmax, tol):
    """Kept values equal the oracle's leading values of each face; columns
    past min(rho_l, kmax) are zero."""
    s = host(out.s)
    U, V = host(out.Uhat), host(out.Vhat)
    for l in range(s.shape[1]):
        kl = min(int(rho[l]), kmax)
        assert rel(s[:kl, l], ref_s_all[:kl, l]) <= tol, l
        assert np.all(s[kl:, l] == 0) and np.all(U[:, kl:, l] == 0) and np.all(V[:, kl:, l] == 0), l


@pytest.mark.parametrize("n1,n2,n3,p,frac", [
    (40, 24, 16, 4, 0.4),      # tall faces
    (24, 40, 16, 4, 0.25),     # wide faces
    (70, 33, 20, 7, 0.6),      # ragged vector count
    (9, 5, 6, 1, 0.5),         # one face
    (300, 260, 40, 24, 0.3),   # 6240 values: several per selection thread
])
def test_svdii_f32(pq, n1, n2, n3, p, frac):
    A, Q = _case(101 + n1, n1, n2, n3, p, np.float32)
    Al = synth.logical(A)
    ref = oracle.tsvdq(Al, Q, 1)
    K = max(1, int(frac * ref.s_all.size))
    gamma = _gamma_between(ref.s_all, K)
    rho_ref, Ak_ref = oracle.tsvdq_ii(Al, Q, gamma)
    assert rho_ref.sum() == K
    say(f"svdii f32 {n1}x{n2}x{n3} p={p} K={K} gamma={gamma:.6f}")
    out = pq.svdii(dev(A), devq(Q.astype(np.float32)), gamma, approx=True)
    assert int(out.info[1].item()) == 0
    rho = out.rho.cpu().numpy()
    np.testing.assert_array_equal(rho, rho_ref)
    _check_factors(out, ref.s_all, rho, min(n1, n2), TOL32)
    e = rel(host(out.Ak), Ak_ref)
    say(f"  rho {rho.tolist()}  Ak rel {e:.2e}")
    assert e <= TOL32


def test_svdii_f64_and_error_identity(pq):
    """The tiny plain-method tensor in float64; the error of the result obeys
    Thm. 4.4 (discarded energy plus the projection error)."""
    c = synth.tiny()
    A, Q = c["A"], c["Q"]
    Al = synth.logical(A)
    ref = oracle.tsvdq(Al, Q, 1)
    K = ref.s_all.size // 3
    gamma = _gamma_between(ref.s_all, K)
    rho_ref, Ak_ref = oracle.tsvdq_ii(Al, Q, gamma)
    out = pq.svdii(dev(A), devq(Q), gamma, approx=True)
    rho = out.rho.cpu().numpy()
    np.testing.assert_array_equal(rho, rho_ref)
    _check_factors(out, ref.s_all, rho, min(Al.shape[:2]), TOL64)
    Ak = host(out.Ak)
    assert rel(Ak, Ak_ref) <= TOL64
    discarded = sum(float(np.sum(ref.s_all[int(rho[l]):, l] ** 2)) for l in range(rho.size))
    projection = oracle.fro2(Al - oracle.proj(Al, Q))
    err2 = oracle.fro2(Al - Ak)
    say(f"svdii f64 tiny: K={K} err2 {err2:.6e} vs {discarded + projection:.6e}")
    assert abs(err2 - (discarded + projection)) <= 1e-9 * err2


def test_svdii_kmax_cap(pq):
    """Faces whose rank exceeds kmax keep kmax triplets; rho is reported
    before the cap and the approximation is the capped sum."""
    n1, n2, n3, p, kmax = 60, 50, 30, 10, 6
    A, Q = _case(7, n1, n2, n3, p, np.float32)
    Al = synth.logical(A)
    full = oracle.tsvdq(Al, Q, min(n1, n2))
    K = int(0.5 * full.s_all.size)
    gamma = _gamma_between(full.s_all, K)
    rho_ref, _ = oracle.tsvdq_ii(Al, Q, gamma)
    assert rho_ref.max() > kmax
    out = pq.svdii(dev(A), devq(Q.astype(np.float32)), gamma, kmax=kmax, approx=True)
    rho = out.rho.cpu().numpy()
    np.testing.assert_array_equal(rho, rho_ref)
    _check_factors(out, full.s_all, rho, kmax, TOL32)
    # the capped approximation from the oracle's factors
    Akh = np.zeros((n1, n2, p))
    for l in range(p):
        kl = min(int(rho[l]), kmax)
        Akh[:, :, l] = (full.Uhat[:, :kl, l] * full.s[:kl, l]) @ full.Vhat[:, :kl, l].T
    Ak_ref = oracle.unhat(Akh, Q)
    assert rel(host(out.Ak), Ak_ref) <= TOL32


def test_svdii_beats_tsvdq(pq):
    """Thm. 4.5 on the GPU's results: with gamma the energy kept by the rank-k
    tSVDQ, SVDII stores no more values and its error is no larger."""
    n1, n2, n3, p, k = 48, 40, 24, 8, 5
    A, Q = _case(19, n1, n2, n3, p, np.float32)
    Ad, Qd = dev(A), devq(Q.astype(np.float32))
    t = pq.tsvdq(Ad, Qd, k, approx=True)
    full = pq.svdii(Ad, Qd, 1.0)
    s_all = host(full.s).astype(np.float64)
    gamma = float(np.sum(s_all[:k] ** 2) / np.sum(s_all ** 2))
    ii = pq.svdii(Ad, Qd, gamma, approx=True)
    rho = ii.rho.cpu().numpy()
    Al = synth.logical(A)
    e_t = np.sqrt(oracle.fro2(Al - host(t.Ak)))
    e_ii = np.sqrt(oracle.fro2(Al - host(ii.Ak)))
    say(f"Thm 4.5: sum rho {rho.sum()} <= {k * p}; error {e_ii:.6e} <= {e_t:.6e}")
    assert rho.sum() <= k * p + 1
    assert e_ii <= e_t * (1 + 1e-6)


def test_svdii_gamma_one_keeps_everything(pq):
    """gamma = 1 keeps every value of nonzero energy: A_k is the projection
    A x_3 Q Q^T (Cor. of Thm. 4.4 with nothing discarded)."""
    A, Q = _case(23, 30, 22, 18, 6, np.float32)
    out = pq.svdii(dev(A), devq(Q.astype(np.float32)), 1.0, approx=True)
    Al = synth.logical(A)
    assert rel(host(out.Ak), oracle.proj(Al, Q)) <= TOL32
    assert np.all(out.rho.cpu().numpy() <= 22)


def test_svdii_compensated_bf16(pq):
    """The split-bfloat16 (x3) transforms keep the selection and the
    approximation within the float32 tolerance."""
    A, Q = _case(29, 64, 48, 40, 12, np.float32)
    Al = synth.logical(A)
    ref = oracle.tsvdq(Al, Q, 1)
    K = int(0.35 * ref.s_all.size)
    gamma = _gamma_between(ref.s_all, K)
    rho_ref, Ak_ref = oracle.tsvdq_ii(Al, Q, gamma)
    out = pq.svdii(dev(A), devq(Q.astype(np.float32)), gamma, prec="bf16x3", approx=True)
    np.testing.assert_array_equal(out.rho.cpu().numpy(), rho_ref)
    assert rel(host(out.Ak), Ak_ref) <= TOL32


def test_svdii_rejects_bad_gamma(pq):
    from paper_2409_19402_amd._lib import ProjProdError
    A, Q = _case(31, 8, 8, 8, 2, np.float32)
    for g in (0.0, -0.5, 1.5, float("nan")):
        with pytest.raises(ProjProdError):
            pq.svdii(dev(A), devq(Q.astype(np.float32)), g)


def test_svdii_video_full_size(pq):
    """The video workload at full size (240 x 320 x 200, p = 20, Q = U3),
    gamma halfway between the cumulative energies around the rank-10 tSVDQ's
    implicit rank."""
    c = synth.video_case()
    Al = synth.logical(c["A"])
    ref = oracle.tsvdq(Al, c["Q"], 1)
    K = 10 * c["Q"].shape[1]
    gamma = _gamma_between(ref.s_all, K)
    rho_ref, Ak_ref = oracle.tsvdq_ii(Al, c["Q"], gamma)
    out = pq.svdii(dev(c["A"]), devq(c["Q"]), gamma, kmax=60, approx=True)
    rho = out.rho.cpu().numpy()
    say(f"svdii video full size: K={K}, rho {rho.tolist()}")
    np.testing.assert_array_equal(rho, rho_ref)
    assert rho_ref.max() <= 60
    assert rel(host(out.Ak), Ak_ref) <= TOL32
    assert relmax(host(out.Ak), Ak_ref) <= 10 * TOL32
