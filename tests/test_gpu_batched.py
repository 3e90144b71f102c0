"""The batched form (pq_batched_plan / pq_batched_run): every instance of an
uneven batch matches the unbatched call on the same inputs and the float64
oracle, on the planning run and on graph replays after the inputs change in
place (with eager work between the replays)."""

import numpy as np
import pytest

import oracle
from helpers import dev, devq, host, rel, relmax, say
from paper_2409_19402_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
# element-wise: max |x - ref| over max |ref|
TOLMAX = 1e-4

# (n1, n2, n3, n4 or None, p, k or None): tall and wide faces, faces of
# fewer than 16 and more than 32 vectors, p = n3, product-only and
# tSVDQ-only instances, odd tube counts (one tube per lane in the grouped
# transforms), a product of more than 32 faces (its back-projection is not
# grouped)
SHAPES = [
    (40, 24, 16, 20, 4, 3),
    (150, 70, 33, 45, 9, 4),
    (12, 90, 20, None, 20, 5),
    (64, 64, 48, 64, 16, 8),
    (33, 130, 24, 17, 7, None),
    (200, 10, 12, 30, 5, 10),
    (37, 21, 40, 29, 36, None),
]


@pytest.fixture(scope="module")
def pq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2409_19402_amd import binding
    return binding


def _inputs(seed):
    rng = np.random.default_rng(seed)
    out = []
    for (n1, n2, n3, n4, p, k) in SHAPES:
        A = synth.gaussian(rng, n1, n2, n3)
        B = synth.gaussian(rng, n2, n4, n3) if n4 else None
        Q = synth.random_orthonormal(rng, n3, p).astype(np.float32)
        out.append(dict(A=A, B=B, Q=Q, k=k))
    return out


def _check(pq, batch, cases, dev_cases, label):
    for i, (c, d, out) in enumerate(zip(cases, dev_cases, batch.outputs)):
        Al = synth.logical(c["A"])
        if c["B"] is not None:
            C_ref = pq.qprod(d["A"], d["B"], d["Q"])
            assert rel(host(out["C"]), host(C_ref)) <= TOL32, (label, i)
            assert rel(host(out["C"]), oracle.qprod(Al, synth.logical(c["B"]), c["Q"])) <= TOL32, (label, i)
        if c["k"] is not None:
            k = c["k"]
            one = pq.tsvdq(d["A"], d["Q"], k)
            assert int(one.info[1].item()) == 0
            ref = oracle.tsvdq(Al, c["Q"], k)
            s = host(out["s"])
            U, V = host(out["Uhat"]), host(out["Vhat"])
            for l in range(s.shape[1]):
                assert rel(s[:, l], ref.s[:, l]) <= TOL32, (label, i, l)
                assert rel(s[:, l], host(one.s)[:, l]) <= TOL32, (label, i, l)
            # the facewise rank-k approximations agree
            approx = np.einsum("ijl,jl,mjl->iml", U, s, V)
            ref_approx = np.einsum("ijl,jl,mjl->iml", ref.Uhat, ref.s, ref.Vhat)
            assert rel(approx, ref_approx) <= TOL32, (label, i)
            say(f"  {label} instance {i}: s rel {rel(s, ref.s):.2e}, approx rel {rel(approx, ref_approx):.2e}")


def test_batched_matches_unbatched_and_replays(pq):
    import torch
    cases = _inputs(11)
    dev_cases = [dict(A=dev(c["A"]), B=None if c["B"] is None else dev(c["B"]), Q=devq(c["Q"]))
                 for c in cases]
    insts = []
    for c, d in zip(cases, dev_cases):
        x = dict(A=d["A"], Q=d["Q"])
        if d["B"] is not None:
            x["B"] = d["B"]
        if c["k"] is not None:
            x["k"] = c["k"]
        insts.append(x)
    say(f"batched plan: {len(insts)} instances")
    batch = pq.batched(insts)
    torch.cuda.synchronize()
    info = batch.info.cpu().tolist()
    say(f"  plan info {info}")
    assert info[1] == 0
    _check(pq, batch, cases, dev_cases, "plan")

    # new data in the same input tensors; replays with eager work between them
    new = _inputs(12)
    for c, d in zip(new, dev_cases):
        d["A"].copy_(dev(c["A"]))
        if c["B"] is not None:
            d["B"].copy_(dev(c["B"]))
        d["Q"].copy_(devq(c["Q"]))
    for rep in range(3):
        for out in batch.outputs:  # clobber the outputs: each replay must rewrite them
            for t in out.values():
                t.fill_(float("nan"))
        batch.run()
        torch.cuda.synchronize()
        assert batch.info.cpu().tolist()[1] == 0
        _check(pq, batch, new, dev_cases, f"replay {rep}")
        _ = pq.hat(dev_cases[0]["A"], dev_cases[0]["Q"])  # eager work between replays
        torch.cuda.synchronize()
    batch.close()


def test_batched_rejects_long_faces(pq):
    from paper_2409_19402_amd._lib import ProjProdError
    rng = np.random.default_rng(3)
    A = dev(synth.gaussian(rng, 600, 8, 8))
    Q = devq(synth.random_orthonormal(rng, 8, 2).astype(np.float32))
    with pytest.raises(ProjProdError):
        pq.batched([dict(A=A, Q=Q, k=2)])


# instances of the full workload compared with the oracle besides every one
# whose faces are longer than 360: the two smallest and two others
FULL_SAMPLE = (17, 23, 42, 62)
GROUPS = 8


@pytest.fixture(scope="module")
def full_batch(pq):
    """The full batched workload (64 uneven instances, n1, n2, n4 up to 512,
    n3 up to 256, p up to 32) planned once; its outputs are clobbered and the
    graph replayed, so every check reads what a replay wrote."""
    import torch
    shapes = synth.batched_shapes(count=64)
    insts = []
    for i, sh in enumerate(shapes):
        c = synth.batched_instance(4, i, sh)
        insts.append(dict(A=dev(c["A"]), B=dev(c["B"]), Q=devq(c["Q"]), k=c["k"]))
    say("batched full config: planning 64 instances")
    batch = pq.batched(insts)
    for out in batch.outputs:
        for t in out.values():
            t.fill_(float("nan"))
    batch.run()
    torch.cuda.synchronize()
    yield shapes, insts, batch
    batch.close()


def test_batched_full_config_converged(full_batch):
    import torch
    shapes, _, batch = full_batch
    info = batch.info.cpu().tolist()
    say(f"  info {info}")
    assert info[1] == 0
    for out in batch.outputs:
        for t in out.values():
            assert bool(torch.isfinite(t).all())


@pytest.mark.parametrize("group", range(GROUPS))
def test_batched_full_config_instances(pq, full_batch, group):
    """Every instance of the full workload against the unbatched calls on the
    same inputs (C = A *_Q B, the singular values and the facewise rank-k
    approximations), and against the float64 oracle for every instance with a
    face longer than 360 plus four others; relative Frobenius norms and
    element-wise maxima."""
    shapes, insts, batch = full_batch
    n = len(shapes)
    for i in range(group * n // GROUPS, (group + 1) * n // GROUPS):
        sh, d, out = shapes[i], insts[i], batch.outputs[i]
        k = sh["k"]
        C = host(out["C"])
        U, s, V = host(out["Uhat"]), host(out["s"]), host(out["Vhat"])
        approx = np.einsum("ijl,jl,mjl->iml", U, s, V)
        one_c = host(pq.qprod(d["A"], d["B"], d["Q"]))
        one = pq.tsvdq(d["A"], d["Q"], k)
        assert int(one.info[1].item()) == 0
        one_s = host(one.s)
        one_a = np.einsum("ijl,jl,mjl->iml", host(one.Uhat), one_s, host(one.Vhat))
        errs = dict(c=rel(C, one_c), cmax=relmax(C, one_c), s=rel(s, one_s), a=rel(approx, one_a),
                    amax=relmax(approx, one_a))
        for l in range(s.shape[1]):
            assert rel(s[:, l], one_s[:, l]) <= TOL32, (i, l)
        line = f"  instance {i} {sh}: vs unbatched " + ", ".join(f"{k2} {v:.1e}" for k2, v in errs.items())
        assert errs["c"] <= TOL32 and errs["s"] <= TOL32 and errs["a"] <= TOL32, line
        assert errs["cmax"] <= TOLMAX and errs["amax"] <= TOLMAX, line
        if max(sh["n1"], sh["n2"]) > 360 or i in FULL_SAMPLE:
            c = synth.batched_instance(4, i, sh)
            Al, Bl = synth.logical(c["A"]), synth.logical(c["B"])
            ref_c = oracle.qprod(Al, Bl, c["Q"])
            ref = oracle.tsvdq(Al, c["Q"], k)
            ref_a = np.einsum("ijl,jl,mjl->iml", ref.Uhat, ref.s, ref.Vhat)
            oe = dict(c=rel(C, ref_c), cmax=relmax(C, ref_c), s=rel(s, ref.s), a=rel(approx, ref_a),
                      amax=relmax(approx, ref_a))
            for l in range(s.shape[1]):
                assert rel(s[:, l], ref.s[:, l]) <= TOL32, (i, l)
            line += "; vs oracle " + ", ".join(f"{k2} {v:.1e}" for k2, v in oe.items())
            assert oe["c"] <= TOL32 and oe["s"] <= TOL32 and oe["a"] <= TOL32, line
            assert oe["cmax"] <= TOLMAX and oe["amax"] <= TOLMAX, line
        say(line)
