"""afm_grad_batch_noalloc (the gradient with its checkpoints in the library's fixed scratch
array, for callers that cannot allocate) against afm_grad_batch through the C ABI: two calls in a
row on one plan, the second with fewer points, each equal to afm_grad_batch's result bit for bit
(the same kernels on the same inputs at the same checkpoint stride); a request larger than the
scratch array is refused before anything is enqueued."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def afm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1109_0334_amd as afm

    afm.lib()
    return afm


def _same(a, b):
    return np.array_equal(a.cpu().numpy().view(np.uint8), b.cpu().numpy().view(np.uint8))


def _case(afm, name, n_cycles, sizes, stride, prec):
    import torch

    c = W.config(name)
    m = dict(c["model"], n_cycles=n_cycles, lockin_cycles=4)
    if name == "c5":
        m["steps_per_cycle"] = 128
    base, free = W.full_params(c), W.free_index(c)
    plan = afm.Plan(m, base, free, precision=prec)
    U = plan.forward_batch(torch.zeros(len(free), 1, dtype=torch.float64, device="cuda")
                           + torch.tensor([[base[f[0]]] for f in free], device="cuda"),
                           trace=True)["trace"]
    for k, n in enumerate(sizes):
        th = torch.tensor(W.draw_free(c, n, 40 + k).T.copy(), device="cuda")
        J0, dJ0, st0 = plan.grad_batch(th, U, ckpt_stride=stride)
        J = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        dJ = torch.full((len(free), n), np.nan, dtype=torch.float64, device="cuda")
        st = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        plan.grad_batch_noalloc(th, U, J, dJ, st, ckpt_stride=stride)
        torch.cuda.synchronize()
        print(f"{name} {prec} n {n} stride {stride}: {int((st0 == 0).sum())} finite")
        assert _same(st, st0) and _same(J, J0) and _same(dJ, dJ0), (name, prec, n)
    plan.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_lj_two_calls_match_grad_batch(afm, prec):
    _case(afm, "c4", 30, (300, 77), 64, prec)


def test_three_modes_default_stride_matches_grad_batch(afm):
    _case(afm, "c5", 12, (130, 9), 0, "mixed")


def test_too_large_is_refused(afm):
    import torch

    c = W.config("c4")
    m = dict(c["model"], n_cycles=1000)
    plan = afm.Plan(m, W.full_params(c), W.free_index(c), precision="mixed")
    n = 4096  # 1000 x 256 / 16 checkpoints x 4 floats x 4096 points > 64 MiB
    th = torch.tensor(W.draw_free(c, n, 49).T.copy(), device="cuda")
    U = torch.zeros(1, plan.W, dtype=torch.float64, device="cuda")
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    dJ = torch.empty(4, n, dtype=torch.float64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(afm.AfmError, match="status 1.*scratch"):
        plan.grad_batch_noalloc(th, U, J, dJ, st, ckpt_stride=16)
    plan.close()
