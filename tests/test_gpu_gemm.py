"""The facewise product of Def. 2.3 on faces large enough for the 128 x 128
matrix-core tiles: every precision mode against a float64 product of the same
faces, element by element, on ragged and aligned shapes."""

import numpy as np
import pytest

from helpers import dev, host, rel, relmax, say
from paper_2409_19402_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOLMAX = 1e-4

# (n1, m, n2, p): ragged in every dimension (scalar loads), aligned (16-byte
# loads), one face, and a face a little over one tile
SHAPES = [
    (130, 97, 257, 3),
    (256, 128, 384, 4),
    (512, 512, 512, 2),
    (129, 300, 128, 1),
    (384, 33, 200, 5),
]


@pytest.fixture(scope="module")
def pq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2409_19402_amd import binding
    return binding


@pytest.mark.parametrize("shape", SHAPES)
def test_facewise_big_tiles(pq, shape):
    n1, m, n2, p = shape
    say(f"facewise big tiles {shape}")
    rng = np.random.default_rng(900 + n1 + m)
    A = synth.gaussian(rng, n1, m, p)
    B = synth.gaussian(rng, m, n2, p)
    ref = np.einsum("irl,rjl->ijl", synth.logical(A).astype(np.float64), synth.logical(B).astype(np.float64))
    Ad, Bd = dev(A), dev(B)
    errs = {}
    for mode in ("default", "bf16x3", "bf16x6", "bf16"):
        C = host(pq.facewise(Ad, Bd, prec=mode))
        errs[mode] = (rel(C, ref), relmax(C, ref))
    say("  " + ", ".join(f"{k} {v[0]:.1e}/{v[1]:.1e}" for k, v in errs.items()))
    for mode in ("default", "bf16x3", "bf16x6"):
        assert errs[mode][0] <= TOL32 and errs[mode][1] <= TOLMAX, (mode, errs[mode])
    # plain bfloat16 is reported; bounded by its unit roundoff times a small factor
    assert errs["bf16"][0] <= 2e-2
