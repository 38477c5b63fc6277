"""Graph replay of one evaluation (pft_evaluate_graph) against the eager calls
(pft_propagate + pft_densities) on the same context: every replay, with the
program's own eager work and synchronisations between replays, reproduces the
eager result bit for bit; new field values at the captured addresses are
used; other buffers are captured anew; the state left behind serves
pft_hamiltonian like an eager evaluation."""
import numpy as np
import pytest
import torch

from paper_1204_5434_amd import binding as B

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, flush=True)


def fields(shape, seed):
    r = np.random.default_rng(seed)
    wp = 0.3 * r.standard_normal(shape) + 0.1j * r.standard_normal(shape)
    wm = 0.3 * r.standard_normal(shape) + 0.1j * r.standard_normal(shape)
    return torch.from_numpy(wp).to(DEV), torch.from_numpy(wm).to(DEV)


CASES = [
    # n, L, ns, f, precision, scheme, model
    ((24, 32, 40), (3.0, 4.0, 5.0), 13, 0.62, B.PFT_C128, B.PFT_RQM4, B.PFT_DIBLOCK),  # axis schedule, junction
    ((16, 24, 24), (2.0, 3.0, 3.0), 20, 0.3, B.PFT_C64, B.PFT_RQM4, B.PFT_DIBLOCK),    # fused yz planes
    ((20, 16, 12), (2.5, 2.0, 1.5), 9, 0.5, B.PFT_C128, B.PFT_SPLIT2, B.PFT_DIBLOCK),
    ((16, 16, 32), (2.0, 2.0, 4.0), 12, 0.5, B.PFT_C64, B.PFT_RQM4, B.PFT_EDWARDS),    # one sweep
]


def make(case):
    n, L, ns, f, prec, scheme, model = case
    return B.Context(B.Params(*n, *L, ns, f, 14.0, 2.0, prec, scheme, model, 1.0 if model == B.PFT_EDWARDS else 0.0))


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-p{c[4]}-s{c[5]}-m{c[6]}" for c in CASES])
def test_graph_replay_matches_eager(case):
    n = case[0]
    ed = case[6] == B.PFT_EDWARDS
    say("graph replay", case)
    ctx = make(case)
    a, b = fields(n, 5)
    a2, b2 = fields(n, 6)
    wm, wm2 = (None, None) if ed else (b, b2)

    def buffers():
        return (torch.empty(n, dtype=torch.complex128, device=DEV), torch.empty(n, dtype=torch.complex128, device=DEV),
                torch.empty(1, dtype=torch.complex128, device=DEV))

    def eager(wp, wmm):
        pa, pb, Q = buffers()
        ctx.pft_propagate(wp, wmm)
        ctx.pft_densities(pa, pb, Q)
        torch.cuda.synchronize()
        return pa, pb, Q

    ref = eager(a, wm)
    ga, gb, gQ = buffers()
    ctx.pft_evaluate_graph(a, wm, ga, gb, gQ, nreps=1)
    torch.cuda.synchronize()
    for x, y in zip((ga, gb, gQ), ref):
        assert torch.equal(x, y)
    for r in range(3):
        # eager work on the same context between replays
        eager(a2, wm2)
        for t in (ga, gb, gQ):
            t.zero_()
        ctx.pft_evaluate_graph(a, wm, ga, gb, gQ, nreps=2)
        torch.cuda.synchronize()
        for x, y in zip((ga, gb, gQ), ref):
            assert torch.equal(x, y), r
    # new values at the captured addresses
    ref2 = eager(a2, wm2)
    a.copy_(a2)
    if not ed:
        b.copy_(b2)
    ctx.pft_evaluate_graph(a, wm, ga, gb, gQ, nreps=1)
    torch.cuda.synchronize()
    for x, y in zip((ga, gb, gQ), ref2):
        assert torch.equal(x, y)
    # the state afterwards serves pft_hamiltonian as after an eager evaluation
    H = torch.empty(1, dtype=torch.complex128, device=DEV)
    ctx.pft_hamiltonian(a, wm, H)
    Hg = H.clone()
    eager(a, wm)
    ctx.pft_hamiltonian(a, wm, H)
    assert torch.equal(H, Hg)
    # other output buffers: captured anew
    ha, hb, hQ = buffers()
    ctx.pft_evaluate_graph(a, wm, ha, hb, hQ, nreps=1)
    torch.cuda.synchronize()
    for x, y in zip((ha, hb, hQ), ref2):
        assert torch.equal(x, y)
    assert ctx.pft_status_flags() == 0
    ctx.close()


def test_graph_replay_rejections():
    n = (16, 16, 16)
    a, b = fields(n, 7)
    pa = torch.empty(n, dtype=torch.complex128, device=DEV)
    pb = torch.empty_like(pa)
    q_only = B.Context(B.Params(*n, 4.0, 4.0, 4.0, 10, 0.5, 14.0, 2.0, B.PFT_C128, B.PFT_RQM4, B.PFT_DIBLOCK, 0.0,
                                B.PFT_STORE_Q))
    with pytest.raises(B.PftError) as e:
        q_only.pft_evaluate_graph(a, b, pa, pb)
    assert e.value.status == B.PFT_E_UNSUPPORTED
    q_only.close()
    ctx = B.Context(B.Params(*n, 4.0, 4.0, 4.0, 10, 0.5, 14.0, 2.0, B.PFT_C128, B.PFT_RQM4))
    with pytest.raises(B.PftError) as e:
        ctx.pft_evaluate_graph(a, b, pa, pb, nreps=-1)
    assert e.value.status == B.PFT_E_INVALID
    ctx.pft_profile_begin()
    with pytest.raises(B.PftError) as e:
        ctx.pft_evaluate_graph(a, b, pa, pb)
    assert e.value.status == B.PFT_E_STATE
    ctx.pft_profile_end()
    ctx.close()
