"""pft_cl_step_static: the field step whose semi-implicit work memory is the
library's fixed device array, for callers that cannot allocate.  Checked
against pft_cl_step on the same inputs (same kernels; the context's own
buffers there): two static calls in a row, the second on a smaller box with
reflecting walls, so it runs on what the first left in the array; both
precisions, diblock and Edwards, semi-implicit and explicit updates; a box
whose work memory exceeds the array is refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_1204_5434_amd import binding as B

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = {B.PFT_C128: 1e-10, B.PFT_C64: 2e-5}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def draw(shape, seed):
    r = np.random.default_rng(seed)
    wp = 0.3 * r.standard_normal(shape) + 0.05j * r.standard_normal(shape)
    wm = 0.4 * r.standard_normal(shape) + 0.05j * r.standard_normal(shape)
    return wp, wm


# (grid, box, ns, walls): the first is the larger input
BOXES = [((64, 48, 40), (6.0, 4.5, 4.0), 24, (0, 0, 0)),
         ((16, 24, 20), (2.0, 3.0, 2.5), 18, (1, 0, 1))]


def step_once(params, wp, wm, st, static):
    ctx = B.Context(params)
    ed = params.model == B.PFT_EDWARDS
    a = dev(wp)
    b = None if ed else dev(wm)
    Q = torch.empty(1, dtype=torch.complex128, device=DEV)
    H = torch.empty_like(Q)
    (ctx.pft_cl_step_static if static else ctx.pft_cl_step)(a, b, st, None, None, Q, H)
    torch.cuda.synchronize()
    out = (host(a), None if ed else host(b), complex(host(Q)[0]), complex(host(H)[0]))
    ctx.close()
    return out


@pytest.mark.parametrize("model", [B.PFT_DIBLOCK, B.PFT_EDWARDS])
@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_static_step_equals_cl_step(prec, model):
    for update in (1, 0):
        for k, (n, L, ns, bc) in enumerate(BOXES):
            params = B.Params(*n, *L, ns, 0.4, 15.0, 20.0, prec, B.PFT_RQM4, model,
                              1.1 if model == B.PFT_EDWARDS else 0.0, B.PFT_STORE_BOTH, bc)
            wp, wm = draw(n, 40 + k)
            st = B.pft_step(0.2, 1.0, 0.6, 77, k, 3, 1, update)
            got = step_once(params, wp, wm, st, True)
            ref = step_once(params, wp, wm, st, False)
            for g, r in zip(got[:2], ref[:2]):
                if r is None:
                    continue
                err = np.abs(g - r).max() / np.abs(r).max()
                print(f"prec {prec} model {model} update {update} box {n} walls {bc}: max rel diff {err:.2e}",
                      flush=True)
                assert err <= TOL[prec]
            assert got[2] == ref[2] and got[3] == ref[3]


def test_static_step_refuses_oversized_work_memory():
    n = (256, 256, 64)   # 4,194,304 sites: 64 MiB for the increment alone
    params = B.Params(*n, 16.0, 16.0, 4.0, 2, 0.5, 15.0, 1.0, B.PFT_C64, B.PFT_SPLIT2)
    ctx = B.Context(params)
    wp = torch.zeros(n, dtype=torch.complex128, device=DEV)
    wm = torch.zeros_like(wp)
    with pytest.raises(B.PftError) as e:
        ctx.pft_cl_step_static(wp, wm, B.pft_step(0.1, 1.0, 1.0, 1, 0, 0, 0, 1))
    assert e.value.status == B.PFT_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert not torch.any(wp != 0) and not torch.any(wm != 0)   # nothing was enqueued
    ctx.close()
