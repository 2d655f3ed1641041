"""GPU: the allocation-free training step (kldi_mlp_step_static, scratch in a static device array)
against the allocating one (kldi_mlp_step) on the same inputs: identical parameters and loss after
each of two calls in a row, the second with a smaller batch; batches beyond the scratch are refused."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_static_step_matches_allocating_step():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_10363_amd import plan as mod
    rng = np.random.default_rng(31)
    theta = (omlp.init_params(rng) + 0.05 * rng.normal(size=omlp.N_PARAMS)).astype(np.float32)
    a, b = mod.Mlp(seed=1), mod.Mlp(seed=1)
    a.params(set_params=theta)
    b.params(set_params=theta)
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for n in (16384, 3001):
        print("case: static step n=%d" % n, flush=True)
        x = torch.from_numpy(rng.uniform(-1, 1, size=(n, 2)).astype(np.float32)).cuda()
        t = torch.from_numpy(rng.normal(size=(n, 3)).astype(np.float32)).cuda()
        La = a.step(x, t, 2e-3)
        b.step_static(x, t, 2e-3, loss=loss)
        torch.cuda.synchronize()
        pa, pb = a.params()[0], b.params()[0]
        print("  loss %.12f vs %.12f, parameters identical: %s" % (La, float(loss.item()), np.array_equal(pa, pb)),
              flush=True)
        assert float(loss.item()) == La
        assert np.array_equal(pa, pb)
        assert not np.array_equal(pa, theta)
    x = torch.zeros((16385, 2), dtype=torch.float32, device="cuda")
    t = torch.zeros((16385, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(mod.L.KldiError) as ei:
        b.step_static(x, t, 2e-3)
    assert ei.value.status == -1 and "16384" in str(ei.value)
    a.close()
    b.close()
