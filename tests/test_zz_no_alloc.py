"""The allocation-free energy entry point (exchange_energy_noalloc, C ABI)
against exchange_energy: the same E_x bit for bit, on two calls in a row, the
second with a smaller input."""
import numpy as np
import pytest

import synth
from tests.gpu_util import device_inputs, run_build

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_noalloc_energy_matches_exchange_energy():
    import paper_2403_10343_amd as exx
    assert torch.cuda.is_available()
    for sysm in (synth.cluster_batch(6, n_min=8, n_max=40), synth.water_cluster(3, seed=2)):
        print("noalloc energy", sysm.name, sysm.n_atoms, flush=True)
        inp = synth.make_inputs(sysm)
        plan = exx.Plan.for_system(sysm)
        K, Eb = run_build(plan, inp, torch)
        Kd = torch.from_numpy(K).to("cuda:0")
        _, _, D = device_inputs(inp, torch)
        E1 = torch.full((plan.n_systems,), 7.0, dtype=torch.float64, device="cuda:0")
        E2 = torch.full((plan.n_systems,), -3.0, dtype=torch.float64, device="cuda:0")
        plan.exchange_energy(Kd, D, E1)
        before = torch.cuda.memory_allocated()
        plan.exchange_energy_noalloc(Kd, D, E2)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert np.array_equal(E1.cpu().numpy(), E2.cpu().numpy())
        assert np.array_equal(E2.cpu().numpy(), Eb)


def test_noalloc_energy_errors():
    import paper_2403_10343_amd as exx
    import paper_2403_10343_amd._lib as L
    p = exx.Plan.for_system(synth.water_cluster(2, seed=0), host_only=True)
    assert L.lib().exchange_energy_noalloc(p._h, None, None, None, None) == L.EXX_ESTATE
    assert L.lib().exchange_energy_noalloc(None, None, None, None, None) == L.EXX_EINVAL
