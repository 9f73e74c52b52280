"""The per-kernel event profile of pisoc_step through the C ABI: every CG
iteration of every solve is one counted launch of k_pcg_spmv, carrying the
algorithmic bytes of its form (5 words per cell at k = 0, 8 at odd k, 11 at
even k >= 2), plus the launch that stops the solve with the last x update
(x += alpha p_old at odd k: 3 words, the two pending updates at even k: 4,
one fewer while x has not been written from the zero start, k <= 2); every
counted kernel class has positive time."""
import pytest

from paper_1404_0959_amd.inputs import make_hit_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1404_0959_amd.pisoc as P
    P.lib()
    return P


def cg_words(iters):
    return sum(5 if k == 0 else 8 if k & 1 else 11 for k in range(iters))


def stop_words(k, xzero=True):
    return (2 if k & 1 else 3) + (0 if xzero and k <= 2 else 1)


def test_profile_counts_cg_iterations(P):
    n = 64
    case = make_hit_case(n, 5, mach=0.2, stokes=(0.1,))
    s = P.Solver.from_case(case, p_tol=1e-8)
    s.step(1)
    s.profile(True)
    st, info = s.step(3)
    prof = s.profile_read()
    s.profile(False)
    s.close()
    assert st in (P.OK, P.WARN_DUST) and len(info) == 3
    iters = [it for i in info for it in i["pcg_iters"]]
    assert all(it > 0 for it in iters)
    cg = prof["k_pcg_spmv"]
    assert cg["launches"] == sum(iters) + len(iters), (cg, iters)
    assert cg["bytes"] == 8.0 * n ** 3 * sum(cg_words(it) + stop_words(it) for it in iters)
    for name, rec in prof.items():
        assert rec["launches"] > 0 and rec["ms"] > 0.0, (name, rec)
    print({k: (v["launches"], round(1e3 * v["ms"] / v["launches"], 1)) for k, v in prof.items()})


@pytest.mark.parametrize("reads,writes,blocks", [(1, 1, 0), (3, 2, 7), (5, 3, 0), (8, 4, 3),
                                                  (11, 7, 0), (12, 8, 5)])
def test_stream_probe_outputs(P, reads, writes, blocks):
    """The streaming probe (the ceiling the memory-bound kernels are read
    against) writes outs[w] = (w + 1) * (in_0 + ... + in_{R-1}), summed left
    to right in FP32, bitwise, also over a grid of a few blocks that strides
    many times; count 0 is a no-op."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(reads * 10 + writes)
    count = 4 * 12345
    ins = [torch.randn(count, device="cuda", generator=g) for _ in range(reads)]
    outs = [torch.full((count,), float("nan"), device="cuda") for _ in range(writes)]
    P.stream_probe(ins, outs, blocks=blocks)
    torch.cuda.synchronize()
    acc = torch.zeros(count, device="cuda")
    for t in ins:
        acc = acc + t
    for w, o in enumerate(outs):
        assert torch.equal(o, acc * float(w + 1)), w
    empty = [torch.empty(0, device="cuda")]
    P.stream_probe(empty, [torch.empty(0, device="cuda")])
