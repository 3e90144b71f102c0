"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: relative Frobenius error <= 1e-5 for float32 results, <= 1e-12
for float64 results, <= 1e-4 for float32 gradients against the float64
reference gradient.  Inputs are seeded and synthetic; the oracle sees exactly
the values the GPU sees (float32 Q and data upcast to float64).
"""

import numpy as np
import pytest

import oracle
from helpers import dev, dev_bf16, devq, host, rel, relmax, say
from paper_2409_19402_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12
# element-wise companion of the float32 norms: max |x - ref| over max |ref|
TOLMAX = 1e-4


@pytest.fixture(scope="module")
def pq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2409_19402_amd import binding
    return binding


def _case(seed, n1, n2, n3, p, dtype=np.float32):
    rng = np.random.default_rng(seed)
    A = synth.gaussian(rng, n1, n2, n3, dtype)
    Q = synth.random_orthonormal(rng, n3, p).astype(dtype)
    return A, Q


TRANSFORM_SHAPES = [
    (32, 24, 16, 4),     # tiny
    (7, 9, 33, 5),       # N = 63: odd tube count, scalar loads, ragged strip
    (50, 30, 200, 20),   # several strips, n3 beyond one 128-row chunk
    (17, 6, 130, 37),    # p > 32: two transform chunks, unhat from global
    (64, 64, 256, 32),   # p = 32 exactly
    (3, 2, 5, 5),        # p = n3
    (1, 1, 9, 3),        # a single tube
]


@pytest.mark.parametrize("shape", TRANSFORM_SHAPES)
def test_transforms_f32(pq, shape):
    n1, n2, n3, p = shape
    say(f"transforms f32 {shape}")
    A, Q = _case(100 + n3, n1, n2, n3, p)
    Ad, Qd = dev(A), devq(Q)
    Al = synth.logical(A)
    Ah = pq.hat(Ad, Qd)
    ref = oracle.hat(Al, Q)
    assert rel(host(Ah), ref) <= TOL32 and relmax(host(Ah), ref) <= TOLMAX
    back = pq.unhat(Ah, Qd)
    ref = oracle.unhat(host(Ah), Q)
    assert rel(host(back), ref) <= TOL32 and relmax(host(back), ref) <= TOLMAX
    P = pq.proj(Ad, Qd)
    ref = oracle.proj(Al, Q)
    assert rel(host(P), ref) <= TOL32 and relmax(host(P), ref) <= TOLMAX


@pytest.mark.parametrize("shape", [(32, 24, 20, 16, 4), (33, 17, 9, 40, 7), (5, 70, 3, 64, 33),
                                   (65, 31, 66, 12, 12)])
def test_qprod_f32(pq, shape):
    n1, m, n2, n3, p = shape
    say(f"qprod f32 {shape}")
    rng = np.random.default_rng(7 + n1)
    A = synth.gaussian(rng, n1, m, n3)
    B = synth.gaussian(rng, m, n2, n3)
    Q = synth.random_orthonormal(rng, n3, p).astype(np.float32)
    C = pq.qprod(dev(A), dev(B), devq(Q))
    ref = oracle.qprod(synth.logical(A), synth.logical(B), Q)
    assert rel(host(C), ref) <= TOL32


def test_facewise_matches_batched_matmul(pq):
    """p = n3 with Q = I: the projected product is the facewise product."""
    say("identity Q")
    rng = np.random.default_rng(21)
    A = synth.gaussian(rng, 40, 30, 8)
    B = synth.gaussian(rng, 30, 50, 8)
    Q = np.eye(8, dtype=np.float32)
    C = host(pq.qprod(dev(A), dev(B), devq(Q)))
    ref = np.einsum("irt,rjt->ijt", synth.logical(A).astype(np.float64),
                    synth.logical(B).astype(np.float64))
    assert rel(C, ref) <= TOL32
    Ch = host(pq.facewise(dev(A), dev(B)))
    assert rel(Ch, ref) <= TOL32


def test_square_orthogonal_roundtrip(pq):
    say("square Q round trip")
    A, Q = _case(5, 20, 12, 24, 24)
    Ad, Qd = dev(A), devq(Q)
    assert rel(host(pq.unhat(pq.hat(Ad, Qd), Qd)), synth.logical(A)) <= TOL32
    assert rel(host(pq.proj(Ad, Qd)), synth.logical(A)) <= TOL32


def test_proj_idempotent(pq):
    say("proj idempotent")
    A, Q = _case(6, 40, 33, 64, 10)
    Qd = devq(Q)
    P1 = pq.proj(dev(A), Qd)
    P2 = pq.proj(P1, Qd)
    assert rel(host(P2), host(P1)) <= TOL32


@pytest.mark.parametrize("shape", [(33, 21, 70, 50, 40), (9, 40, 17, 300, 8), (64, 16, 80, 24, 24)])
def test_transforms_and_qprod_f64(pq, shape):
    """float64 transforms (p up to 40: several column groups per grid row)
    and the float64 facewise product on MFMA tiles of both widths."""
    n1, m, n2, n3, p = shape
    say(f"f64 transforms and qprod {shape}")
    rng = np.random.default_rng(13 + n1)
    A = synth.gaussian(rng, n1, m, n3, np.float64)
    B = synth.gaussian(rng, m, n2, n3, np.float64)
    Q = synth.random_orthonormal(rng, n3, p)
    Al, Bl = synth.logical(A), synth.logical(B)
    assert rel(host(pq.hat(dev(A), devq(Q))), oracle.hat(Al, Q)) <= TOL64
    C = pq.qprod(dev(A), dev(B), devq(Q))
    assert rel(host(C), oracle.qprod(Al, Bl, Q)) <= TOL64


def test_f64_tiny_case(pq):
    """Tiny plain-method case in float64: qprod and tSVDQ (k=5)."""
    say("tiny f64")
    import torch
    c = synth.tiny()
    A, B, Q, k = c["A"], c["B"], c["Q"], c["k"]
    Ad, Bd, Qd = dev(A), dev(B), devq(Q)
    C = pq.qprod(Ad, Bd, Qd)
    assert C.dtype == torch.float64
    assert rel(host(C), oracle.qprod(synth.logical(A), synth.logical(B), Q)) <= TOL64
    r = pq.tsvdq(Ad, Qd, k, spatial=True, approx=True)
    ref = oracle.tsvdq(synth.logical(A), Q, k)
    assert rel(host(r.s), ref.s) <= TOL64
    assert rel(host(r.Ak), ref.Ak) <= 1e-11
    # spatial factors (Alg. 4.1 step 4): S_k is sign-free; U_k and V_k are
    # checked as the transform of the GPU's own transform-domain factors
    ref_sk = np.stack([np.diagonal(ref.Sk[:, :, t]) for t in range(16)], axis=1)
    assert rel(host(r.Sk), ref_sk) <= 1e-11
    assert rel(host(r.Uk), oracle.unhat(host(r.Uhat), Q)) <= TOL64
    assert rel(host(r.Vk), oracle.unhat(host(r.Vhat), Q)) <= TOL64
    info = r.info.cpu().numpy()
    assert info[1] == 0 and 1 <= info[0] <= 30


def _check_tsvdq(pq, A_st, Q, k, tol_s=TOL32, tol_a=TOL32, a_dev=None):
    Al = synth.logical(A_st)
    Ad = dev(A_st) if a_dev is None else a_dev
    r = pq.tsvdq(Ad, devq(Q), k, spatial=True, approx=True)
    info = r.info.cpu().numpy()
    say(f"  jacobi info (max sweeps, unconverged, total) = {info.tolist()}")
    assert info[1] == 0, f"unconverged faces: {info}"
    ref = oracle.tsvdq(Al, Q, k)
    s = host(r.s)
    p = Q.shape[1]
    for l in range(p):
        assert rel(s[:, l], ref.s[:, l]) <= tol_s, f"face {l}"
    assert rel(host(r.Ak), ref.Ak) <= tol_a
    assert relmax(host(r.Ak), ref.Ak) <= 10 * tol_a
    Uh, Vh = host(r.Uhat), host(r.Vhat)
    Ah = oracle.hat(Al, Q)
    for l in range(p):
        nz = s[:, l] > 0
        U = Uh[:, nz, l]
        V = Vh[:, nz, l]
        # both factors orthonormal to working precision (Def. 3.4 in the
        # transform domain: each face of Uhat and Vhat has orthonormal columns)
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=2e-6)
        np.testing.assert_allclose(V.T @ V, np.eye(V.shape[1]), atol=2e-6)
        # U^T Ah = diag(s) V^T on every face
        lhs = U.T @ Ah[:, :, l]
        rhs = s[nz, l][:, None] * Vh[:, nz, l].T
        assert rel(lhs, rhs) <= 10 * tol_a
    # Thm 4.2 from the GPU's own outputs
    ey, pe = oracle.tsvdq_error_terms(Al, Q, k, s_all=ref.s_all)
    err2 = oracle.fro2(Al - host(r.Ak))
    assert abs(err2 - (ey + pe)) <= 1e-4 * (ey + pe) + 1e-6 * oracle.fro2(Al)
    return r, ref


@pytest.mark.parametrize("shape", [(32, 24, 16, 4, 5), (24, 40, 20, 6, 3), (50, 50, 12, 3, 50),
                                   (70, 9, 30, 5, 1), (9, 70, 30, 5, 9), (129, 65, 40, 7, 8),
                                   (1100, 8, 10, 3, 4), (1, 17, 6, 2, 1)])
def test_tsvdq_f32(pq, shape):
    n1, n2, n3, p, k = shape
    say(f"tsvdq f32 {shape}")
    A, Q = _case(300 + n1, n1, n2, n3, p)
    _check_tsvdq(pq, A, Q, k)


def test_tsvdq_f64_blocked(pq):
    """float64 faces large enough to need several block pairs per sweep."""
    say("tsvdq f64 blocked")
    A, Q = _case(77, 70, 40, 12, 3, np.float64)
    Al = synth.logical(A)
    r = pq.tsvdq(dev(A), devq(Q), 5, approx=True)
    ref = oracle.tsvdq(Al, Q, 5)
    assert rel(host(r.s), ref.s) <= TOL64
    assert rel(host(r.Ak), ref.Ak) <= 1e-11
    assert r.info.cpu().numpy()[1] == 0


def test_tsvdq_nonfinite_input_returns(pq):
    """A NaN in the data reaches every face through the transform; the call
    still returns (every sweep loop is bounded and a NaN never requests a
    rotation), with the sweep counts inside their caps and NaN values out."""
    import torch
    say("tsvdq with a NaN")
    A, Q = _case(12, 40, 30, 16, 4)
    A = A.copy()
    A[3, 5, 7] = np.nan  # storage (n3, n2, n1)
    r = pq.tsvdq(dev(A), devq(Q), 3, approx=True)
    torch.cuda.synchronize()
    info = r.info.cpu().numpy()
    assert 0 <= info[0] <= 16 and 0 <= info[1] <= 4
    assert not np.all(np.isfinite(host(r.s)))


def test_tsvdq_rank_deficient(pq):
    """Example 4.1 with the Haar column: the transform face is rank one, so the
    second singular vector of each side must come back as zeros, and the error
    is the printed 0 + 2."""
    say("tsvdq rank deficient")
    import torch
    A = np.zeros((2, 2, 2))
    A[:, :, 0] = [[1, 0], [0, 1]]
    A[:, :, 1] = [[1, 0], [0, -1]]
    Q = (np.array([[1.0], [1.0]]) / np.sqrt(2.0))
    r = pq.tsvdq(dev(synth.storage(A)), devq(Q), 2, approx=True)
    s = host(r.s)
    assert s[0, 0] == pytest.approx(np.sqrt(2.0), rel=1e-14) and s[1, 0] == 0.0
    assert np.all(host(r.Uhat)[:, 1, 0] == 0) and np.all(host(r.Vhat)[:, 1, 0] == 0)
    assert oracle.fro2(A - host(r.Ak)) == pytest.approx(2.0, abs=1e-12)
    assert r.Ak.dtype == torch.float64


def test_tsvdq_split_sweeps_and_graph_replay(pq):
    """32 faces of 512 x 512 hold two visits per CU in a sweep launch, so the
    float32 sweeps run the two halves of the face range on two streams: the
    result against the oracle, and a captured graph of the same call (the
    fork and join captured as graph dependencies) replayed three times with
    eager work between replays, each replay equal to the eager call."""
    import torch
    say("tsvdq split sweeps 512x512x32, p=32, and a captured graph")
    A, Q = _case(41, 512, 512, 32, 32)
    Ad, Qd = dev(A), devq(Q)
    k = 4
    r0 = pq.tsvdq(Ad, Qd, k, approx=True)
    torch.cuda.synchronize()
    assert r0.info.cpu().numpy()[1] == 0
    ref = oracle.tsvdq(synth.logical(A), Q, k)
    assert rel(host(r0.s), ref.s) <= TOL32
    assert rel(host(r0.Ak), ref.Ak) <= TOL32
    s0, ak0 = r0.s.clone(), r0.Ak.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pq.tsvdq(Ad, Qd, k, approx=True)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r1 = pq.tsvdq(Ad, Qd, k, approx=True)
    for rep in range(3):
        junk = torch.randn(1 << 20, device=Ad.device).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"  replay {rep}: max |s - s_eager| = {(r1.s - s0).abs().max().item():.3e}")
        assert torch.equal(r1.s, s0), f"replay {rep}: s differs"
        assert torch.equal(r1.Ak, ak0), f"replay {rep}: A_k differs"
        del junk


def test_tsvdq_max_sweeps_reported(pq):
    """max_sweeps caps each phase (float32 sweeps, then float64 polishing);
    faces stopped by the cap are counted and their outputs still written."""
    say("tsvdq max_sweeps=1")
    A, Q = _case(9, 40, 30, 12, 3)
    r = pq.tsvdq(dev(A), devq(Q), 4, max_sweeps=1)
    info = r.info.cpu().numpy()
    assert info[0] == 2 and info[1] == 3 and info[2] == 6
    assert np.all(np.isfinite(host(r.s)))


def test_video_case_full_size(pq):
    """Video-shaped tSVDQ at 240 x 320 x 200, p = 20, k = 10 (float32)."""
    say("video case 240x320x200")
    c = synth.video_case()
    r, ref = _check_tsvdq(pq, c["A"], c["Q"], c["k"])
    re_gpu = oracle.relative_error(synth.logical(c["A"]), host(r.Ak))
    re_ref = oracle.relative_error(synth.logical(c["A"]), ref.Ak)
    say(f"  RE gpu {re_gpu:.6e}  oracle {re_ref:.6e}")
    assert abs(re_gpu - re_ref) <= 1e-5 * re_ref


def test_hyperspectral_hat_bf16_input(pq):
    """bfloat16-stored hyperspectral cube (512 x 512 x 224, p = 32): float32
    transform of the exact bfloat16 values."""
    say("hyperspectral hat bf16 input")
    c = synth.hyperspectral_case()
    Ad = dev_bf16(c["A_bits"])
    Ah = pq.hat(Ad, devq(c["Q"]))
    ref = oracle.hat(synth.logical(c["A"]), c["Q"])
    assert rel(host(Ah), ref) <= TOL32
    assert relmax(host(Ah), ref) <= TOLMAX


BF16_SHAPES = [(32, 24, 16, 4), (7, 9, 33, 5), (50, 30, 200, 20), (17, 6, 300, 37),
               (64, 64, 256, 32)]


@pytest.mark.parametrize("shape", BF16_SHAPES)
def test_hat_bf16_modes_f32_input(pq, shape):
    """bfloat16 matrix-core transform of float32 data: split x3 and x6 meet
    the float32 tolerance; plain bfloat16 is reported (bounded loosely)."""
    n1, n2, n3, p = shape
    say(f"hat bf16 modes {shape}")
    A, Q = _case(500 + n3, n1, n2, n3, p)
    Ad, Qd = dev(A), devq(Q)
    ref = oracle.hat(synth.logical(A), Q)
    errs = {m: rel(host(pq.hat(Ad, Qd, prec=m)), ref) for m in ("bf16", "bf16x3", "bf16x6")}
    say(f"  rel err {errs}")
    assert errs["bf16x3"] <= TOL32
    assert errs["bf16x6"] <= 1e-6
    assert errs["bf16"] <= 1e-2


@pytest.mark.parametrize("shape", BF16_SHAPES[:3])
def test_hat_bf16_modes_bf16_input(pq, shape):
    """bfloat16-stored data: with Q split three ways the products are exact in
    float32, so split modes meet float32 accuracy."""
    n1, n2, n3, p = shape
    say(f"hat bf16-input modes {shape}")
    A, Q = _case(600 + n3, n1, n2, n3, p)
    bits = synth.bf16_bits(A)
    vals = synth.bf16_to_f32(bits)
    Ad = dev_bf16(bits)
    ref = oracle.hat(synth.logical(vals), Q)
    for m, tol in (("default", TOL32), ("bf16x3", 1e-6), ("bf16x6", 1e-6), ("bf16", 1e-2)):
        assert rel(host(pq.hat(Ad, devq(Q), prec=m)), ref) <= tol, m


@pytest.fixture(scope="module")
def hyper_case():
    c = synth.hyperspectral_case()
    c["ref"] = oracle.tsvdq(synth.logical(c["A"]), c["Q"], c["k"])
    return c


@pytest.mark.parametrize("prec", ["default", "bf16x3"])
def test_hyperspectral_tsvdq(pq, hyper_case, prec):
    """Hyperspectral-shaped case at full size (512 x 512 x 224 bfloat16, p = 32,
    k = 16; flat spectra at the truncation): singular values and A_k against
    the float64 oracle, through the float32 and the split-bfloat16 transform."""
    say(f"hyperspectral tsvdq {prec}")
    c = hyper_case
    Ad = dev_bf16(c["A_bits"])
    Q, k = c["Q"], c["k"]
    r = pq.tsvdq(Ad, devq(Q), k, prec=prec, approx=True)
    info = r.info.cpu().numpy()
    say(f"  jacobi info {info.tolist()}")
    assert info[1] == 0
    ref = c["ref"]
    s = host(r.s)
    for l in range(Q.shape[1]):
        assert rel(s[:, l], ref.s[:, l]) <= TOL32, f"face {l}"
    err = rel(host(r.Ak), ref.Ak)
    errmax = relmax(host(r.Ak), ref.Ak)
    say(f"  A_k rel err {err:.3e}, element-wise {errmax:.3e}")
    assert err <= TOL32
    assert errmax <= TOLMAX


def test_differentiation_case(pq):
    """Gradients of ||A *_Q B - T||^2 at 256x128x128 * 128x256x128, p = 16,
    against the float64 reference gradient; dQ is deterministic."""
    say("differentiation case")
    import torch
    c = synth.differentiation_case()
    A, B, Q, T = c["A"], c["B"], c["Q"], c["T"]
    Ad = dev(A).requires_grad_(True)
    Bd = dev(B).requires_grad_(True)
    Qd = devq(Q).requires_grad_(True)
    Td = dev(T)
    C = pq.qprod(Ad, Bd, Qd)
    loss = ((C - Td) ** 2).sum()
    loss.backward()
    Al, Bl, Tl = synth.logical(A), synth.logical(B), synth.logical(T)
    Cref = oracle.qprod(Al, Bl, Q)
    assert rel(host(C), Cref) <= TOL32
    assert relmax(host(C), Cref) <= TOLMAX
    dA, dB, dQ = oracle.qprod_backward(2 * (Cref - Tl), Al, Bl, Q)
    for got, want in ((Ad.grad, dA), (Bd.grad, dB), (Qd.grad, dQ)):
        assert rel(host(got), want) <= 1e-4
        assert relmax(host(got), want) <= 1e-3
    # fixed-order split-K reduction: bit-identical on repetition
    G = pq.from_storage(torch.from_numpy(np.ascontiguousarray(
        synth.storage(2 * (host(C) - Tl)).astype(np.float32))).cuda())
    r1 = pq.qprod_backward(G, Ad.detach(), Bd.detach(), Qd.detach())
    r2 = pq.qprod_backward(G, Ad.detach(), Bd.detach(), Qd.detach())
    for x, y in zip(r1, r2):
        assert torch.equal(x, y)


@pytest.mark.parametrize("shape", [(20, 70, 130, 90, 24), (7, 33, 97, 130, 5), (32, 128, 256, 200, 32)])
def test_qprod_backward_narrow_outputs(pq, shape):
    """Products whose outputs have at most 32 rows and more than 64 columns
    (the facewise product and dA-hat of thin faces, the dQ products), on
    aligned and unaligned sizes, forward and backward."""
    n1, m, n2, n3, p = shape
    say(f"qprod backward narrow {shape}")
    rng = np.random.default_rng(91 + n1)
    A = synth.gaussian(rng, n1, m, n3)
    B = synth.gaussian(rng, m, n2, n3)
    G = synth.gaussian(rng, n1, n2, n3)
    Q = synth.random_orthonormal(rng, n3, p).astype(np.float32)
    Al, Bl, Gl = synth.logical(A), synth.logical(B), synth.logical(G)
    C = pq.qprod(dev(A), dev(B), devq(Q))
    assert rel(host(C), oracle.qprod(Al, Bl, Q)) <= TOL32
    dA, dB, dQ = pq.qprod_backward(dev(G), dev(A), dev(B), devq(Q))
    ref = oracle.qprod_backward(Gl, Al, Bl, Q)
    for got, want in zip((dA, dB, dQ), ref):
        assert rel(host(got), want) <= 1e-4


@pytest.mark.parametrize("shape", [(1, 1, 1), (33, 17, 65), (64, 32, 128), (5, 300, 7)])
def test_relayout(pq, shape):
    """numpy C order (tube-major) <-> the paper's face-major order, every
    dtype, bit-exact both ways; a C-order gradient goes through it."""
    import torch
    say(f"relayout {shape}")
    rng = np.random.default_rng(sum(shape))
    X = torch.from_numpy(rng.standard_normal(shape)).cuda()
    for dt in (torch.float32, torch.float64, torch.bfloat16):
        Xd = X.to(dt).contiguous()
        F = pq.to_face_major(Xd)
        assert pq.is_face_major(F) and torch.equal(F, Xd)
        T = pq.to_tube_major(F)
        assert T.is_contiguous() and torch.equal(T, Xd)
        assert torch.equal(pq._face_major(Xd), Xd)


def test_proj_backward(pq):
    say("proj backward")
    A, Q = _case(44, 30, 20, 48, 6)
    rng = np.random.default_rng(45)
    T = synth.gaussian(rng, 30, 20, 48)
    Ad = dev(A).requires_grad_(True)
    Qd = devq(Q).requires_grad_(True)
    P = pq.proj(Ad, Qd)
    ((P - dev(T)) ** 2).sum().backward()
    Al, Tl = synth.logical(A), synth.logical(T)
    G = 2 * (oracle.proj(Al, Q) - Tl)
    dA, dQ = oracle.proj_backward(G, Al, Q)
    assert rel(host(Ad.grad), dA) <= 1e-4
    assert rel(host(Qd.grad), dQ) <= 1e-4


def test_f64_gradients(pq):
    say("f64 gradients")
    c = synth.tiny()
    A, B, Q = c["A"], c["B"], c["Q"]
    rng = np.random.default_rng(3)
    G = rng.standard_normal((16, 20, 32))
    dA, dB, dQ = pq.qprod_backward(dev(G), dev(A), dev(B), devq(Q))
    ref = oracle.qprod_backward(synth.logical(G), synth.logical(A), synth.logical(B), Q)
    assert rel(host(dA), ref[0]) <= TOL64
    assert rel(host(dB), ref[1]) <= TOL64
    assert rel(host(dQ), ref[2]) <= TOL64


def test_check_q(pq):
    say("check_q")
    import torch
    Q = synth.random_orthonormal(np.random.default_rng(1), 200, 20)
    assert pq.check_q(devq(Q)).item() == pytest.approx(oracle.check_q(Q), abs=1e-15)
    Qp = Q.copy()
    Qp[3, 2] += 1e-3
    assert pq.check_q(devq(Qp)).item() == pytest.approx(oracle.check_q(Qp), rel=1e-12)
    Q32 = Q.astype(np.float32)
    assert pq.check_q(devq(Q32)).item() == pytest.approx(oracle.check_q(Q32), rel=1e-9, abs=1e-15)
    assert pq.check_q(devq(Q32)).dtype == torch.float64


def test_autotuned_launches_match(pq, tmp_path):
    """Every candidate configuration the autotuner may pick computes the same
    transform: results with tuning on and off agree, and the table persists."""
    say("autotune")
    from paper_2409_19402_amd import _lib
    A, Q = _case(71, 45, 37, 70, 9)
    Ad, Qd = dev(A), devq(Q)
    ref = oracle.hat(synth.logical(A), Q)
    pq.autotune(True)
    try:
        tuned = {m: host(pq.hat(Ad, Qd, prec=m)) for m in ("default", "bf16x3")}
        P = host(pq.proj(Ad, Qd))
    finally:
        pq.autotune(False)
    assert rel(tuned["default"], ref) <= TOL32
    assert rel(tuned["bf16x3"], ref) <= TOL32
    assert rel(P, oracle.proj(synth.logical(A), Q)) <= TOL32
    n = _lib.load().pq_autotune_entries()
    assert n >= 3
    path = tmp_path / "tune.txt"
    pq.autotune_save(path)
    assert len(path.read_text().splitlines()) == n
    pq.autotune_load(path)
    assert _lib.load().pq_autotune_entries() == n


def test_rejects_non_face_major(pq):
    import torch
    X = torch.zeros((4, 5, 6), device="cuda")  # C-contiguous, not face-major
    Q = torch.zeros((6, 2), device="cuda")
    with pytest.raises(ValueError):
        pq.hat(X, Q)


@pytest.mark.parametrize("shape", [(50, 30, 200, 20), (7, 9, 33, 5), (64, 64, 256, 32)])
def test_proj_fused_without_workspace(pq, shape):
    """pq_proj with no workspace runs the fused single-pass kernel (p <= 32)."""
    import ctypes
    from paper_2409_19402_amd import _lib
    n1, n2, n3, p = shape
    say(f"proj fused {shape}")
    A, Q = _case(300 + n3, n1, n2, n3, p)
    Ad, Qd = dev(A), devq(Q)
    out = pq.empty(n1, n2, n3, device=Ad.device)
    import torch
    s = torch.cuda.current_stream().cuda_stream
    _lib.call("pq_proj", Ad.data_ptr(), 0, Qd.data_ptr(), out.data_ptr(), n1, n2, n3, p, 0, None, 0, s)
    assert rel(host(out), oracle.proj(synth.logical(A), Q)) <= TOL32
    # and it refuses p > 32 without a workspace
    A2, Q2 = _case(301, 8, 8, 40, 33)
    out2 = pq.empty(8, 8, 40, device=Ad.device)
    with pytest.raises(_lib.ProjProdError):
        _lib.call("pq_proj", dev(A2).data_ptr(), 0, devq(Q2).data_ptr(), out2.data_ptr(), 8, 8, 40, 33, 0,
                  None, 0, s)


FACEWISE_SHAPES = [(64, 128, 64, 4), (33, 17, 9, 3), (100, 300, 70, 2), (256, 128, 256, 4)]


@pytest.mark.parametrize("shape", FACEWISE_SHAPES)
def test_facewise_modes(pq, shape):
    """Facewise product (Def. 2.3) in every precision mode: float32 and the
    split-bfloat16 forms meet the float32 tolerance (x6 a tighter one); plain
    bfloat16 is reported and loosely bounded."""
    n1, m, n2, p = shape
    rng = np.random.default_rng(900 + n1)
    Ah = synth.gaussian(rng, n1, m, p)
    Bh = synth.gaussian(rng, m, n2, p)
    ref = oracle.facewise(synth.logical(Ah), synth.logical(Bh))
    errs = {}
    for mode in ("default", "bf16x3", "bf16x6", "bf16"):
        errs[mode] = rel(host(pq.facewise(dev(Ah), dev(Bh), prec=mode)), ref)
    say(f"facewise {shape}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert errs["default"] <= TOL32
    assert errs["bf16x3"] <= TOL32
    assert errs["bf16x6"] <= 1e-6
    assert errs["bf16"] <= 1e-2


@pytest.mark.parametrize("shape", [(32, 24, 20, 16, 4), (65, 31, 66, 12, 12), (128, 64, 128, 64, 16)])
def test_qprod_modes(pq, shape):
    """The whole product in the compensated modes (transform and facewise
    product split, back-projection float32) against the float64 oracle."""
    n1, m, n2, n3, p = shape
    rng = np.random.default_rng(70 + n1)
    A = synth.gaussian(rng, n1, m, n3)
    B = synth.gaussian(rng, m, n2, n3)
    Q = synth.random_orthonormal(rng, n3, p).astype(np.float32)
    ref = oracle.qprod(synth.logical(A), synth.logical(B), Q)
    errs = {mode: rel(host(pq.qprod(dev(A), dev(B), devq(Q), prec=mode)), ref)
            for mode in ("bf16x3", "bf16x6", "bf16")}
    say(f"qprod modes {shape}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert errs["bf16x3"] <= TOL32
    assert errs["bf16x6"] <= 1e-6
    assert errs["bf16"] <= 1e-2


@pytest.mark.parametrize("shape", [(50, 30, 200, 20), (7, 9, 33, 5), (64, 64, 256, 32), (17, 6, 300, 37)])
def test_unhat_modes(pq, shape):
    """Back-projection in every precision mode (p > 32 falls back to float32)."""
    n1, n2, n3, p = shape
    rng = np.random.default_rng(950 + n3)
    Ah = synth.gaussian(rng, n1, n2, p)
    Q = synth.random_orthonormal(rng, n3, p).astype(np.float32)
    ref = oracle.unhat(synth.logical(Ah), Q)
    errs = {mode: rel(host(pq.unhat(dev(Ah), devq(Q), prec=mode)), ref)
            for mode in ("default", "bf16x3", "bf16x6", "bf16")}
    say(f"unhat {shape}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert errs["default"] <= TOL32
    assert errs["bf16x3"] <= TOL32
    assert errs["bf16x6"] <= 1e-6
    assert errs["bf16"] <= 1e-2
