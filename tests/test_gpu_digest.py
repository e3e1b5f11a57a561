"""f12_digest (chunk checksum of streamed output) against the host definition:
integral blocks of the 3-atom molecule, random bit patterns over a list large
enough for the grid-stride loop (more than 4096 work-groups' worth), chunked
ranges adding up to the whole, empty ranges and argument errors."""
import numpy as np
import pytest

from synth import FACTOR_SETS, molecule, tiny_config
from tests.digest_ref import digest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_5070_amd import f12int
    return f12int


def _u64(t):
    return int(t.cpu().numpy().view(np.uint64)[0])


def test_digest_of_integral_blocks(lib):
    import torch
    _, shells = tiny_config()
    pairs = lib.Pairs(lib.Basis.from_shells(shells), 0)
    P1 = FACTOR_SETS["P1"]
    k = lib.Kernel(3, P1, P1)
    Q = lib.Quartets.build(pairs, pairs, 3)
    out = torch.empty(Q.n_out, dtype=torch.float64, device="cuda")
    lib.eval_into(Q, k, out)
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    lib.digest(Q, out, d)
    lib.stream_status()
    assert _u64(d) == digest(out.cpu().numpy())
    # chunks: each digested from a buffer holding only its own blocks
    offs = Q.offsets()
    cuts = [0, 1, Q.n_quartets // 3, Q.n_quartets - 1, Q.n_quartets]
    dc = torch.zeros(1, dtype=torch.int64, device="cuda")
    for a, b in zip(cuts[:-1], cuts[1:]):
        part = out[int(offs[a]):int(offs[b])].clone()
        lib.digest(Q, part, dc, a, b)
    lib.stream_status()
    assert _u64(dc) == _u64(d)


def test_digest_large_range(lib):
    import torch
    # one (ff|ff) quartet repeated: 10,000 doubles per block, 4.4e6 doubles in all
    _, fsh = molecule(11, 2, 3.0, 0.0, (3,), 2, 2, 0.3, 3.0)
    pairs = lib.Pairs(lib.Basis.from_shells(fsh), 1)
    quads = [(0, 1, 0, 1)] * 440
    Q = lib.Quartets.from_list(pairs, pairs, 3, quads)
    assert Q.n_out == 440 * 10 ** 4
    g = torch.Generator(device="cuda").manual_seed(5)
    bits = torch.randint(-2 ** 62, 2 ** 62, (Q.n_out,), dtype=torch.int64, device="cuda", generator=g)
    x = bits.view(torch.float64)
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    lib.digest(Q, x, d)
    dc = torch.full((1,), 12345, dtype=torch.int64, device="cuda")  # accumulates onto the value given
    lib.digest(Q, x[:10 ** 4 * 101], dc, 0, 101)
    lib.digest(Q, x[10 ** 4 * 101:], dc, 101, 440)
    lib.stream_status()
    ref = digest(x.cpu().numpy())
    assert _u64(d) == ref
    assert _u64(dc) == (ref + 12345) % 2 ** 64


def test_digest_empty_and_errors(lib):
    import torch
    _, shells = tiny_config()
    pairs = lib.Pairs(lib.Basis.from_shells(shells), 1)
    Q = lib.Quartets.from_list(pairs, pairs, 3, [(0, 0, 0, 0), (1, 0, 1, 0)])
    out = torch.zeros(Q.n_out, dtype=torch.float64, device="cuda")
    d = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    lib.digest(Q, out, d, 1, 1)
    lib.stream_status()
    assert _u64(d) == 7
    for a, b in ((-1, 1), (0, 3), (2, 1)):
        with pytest.raises(RuntimeError):
            lib.digest(Q, out, d, a, b)
