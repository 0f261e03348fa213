"""Two Coulomb matrices in one call (build_K_two_kernels) against the CPU
oracle, and against build_K on each Coulomb matrix."""
import numpy as np
import pytest

import synth
from oracle import exx_oracle as O
from tests.gpu_util import device_inputs, relmax, system_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_K = 1e-10
TOL_E = 1e-10


@pytest.fixture(scope="module")
def exx():
    import paper_2403_10343_amd as m
    assert torch.cuda.is_available()
    return m


def two_build(plan, inp, V2, precision=0):
    dev = "cuda:0"
    C, V, D = device_inputs(inp, torch)
    V2d = torch.from_numpy(np.ascontiguousarray(V2)).to(dev)
    n = plan.info["d_size"]
    K2 = torch.empty(2 * n, dtype=torch.float64, device=dev)
    Ex = torch.empty(2 * plan.n_systems, dtype=torch.float64, device=dev)
    plan.build_K_two_kernels(C, V, V2d, D, K2, Ex, precision=precision)
    torch.cuda.synchronize()
    return K2.cpu().numpy().reshape(2, n), Ex.cpu().numpy().reshape(2, plan.n_systems)


def one_build(plan, inp, Vx, precision=0):
    dev = "cuda:0"
    C, _, D = device_inputs(inp, torch)
    Vd = torch.from_numpy(np.ascontiguousarray(Vx)).to(dev)
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device=dev)
    Ex = torch.empty(plan.n_systems, dtype=torch.float64, device=dev)
    plan.build_K(C, Vd, D, K, Ex, precision=precision)
    torch.cuda.synchronize()
    return K.cpu().numpy(), Ex.cpu().numpy()


@pytest.mark.parametrize("n_mol,seed", [(1, 6), (2, 7), (8, 8)])
def test_two_kernels_clusters_match_oracle(exx, n_mol, seed):
    sysm = synth.water_cluster(n_mol, seed)
    print("two kernels cluster", n_mol, flush=True)
    inp = synth.make_inputs(sysm)
    V2 = synth.short_range_V(inp)
    K2, Ex = two_build(exx.Plan.for_system(sysm), inp, V2)
    Ko = O.k_two_kernels(inp, V2)
    Dm = O.Blocks(inp).D
    for a in range(2):
        Kg = system_block(K2[a], inp.layout, 0)
        assert relmax(Kg, Ko[a]) < TOL_K
        assert np.array_equal(Kg, Kg.T)
        Eo = O.exchange_energy(Ko[a], Dm)
        assert abs(Ex[a, 0] - Eo) < TOL_E * abs(Eo)


def test_two_kernels_config1_4index(exx):
    inp = synth.make_inputs(synth.config(1))
    V2 = synth.short_range_V(inp)
    K2, Ex = two_build(exx.Plan.for_system(inp.system), inp, V2)
    Ko = O.k_two_kernels(inp, V2, route="4index")
    for a in range(2):
        assert relmax(system_block(K2[a], inp.layout, 0), Ko[a]) < TOL_K


def test_two_kernels_uneven_batch(exx):
    sysm = synth.cluster_batch(4, batch_seed=9, n_min=2, n_max=12)
    print("two kernels batch", sysm.n_systems, flush=True)
    inp = synth.make_inputs(sysm)
    V2 = synth.short_range_V(inp)
    K2, Ex = two_build(exx.Plan.for_system(sysm), inp, V2)
    for c in range(sysm.n_systems):
        Ko = O.k_two_kernels(inp, V2, s=c)
        Dm = system_block(inp.D, inp.layout, c)
        for a in range(2):
            assert relmax(system_block(K2[a], inp.layout, c), Ko[a]) < TOL_K
            Eo = O.exchange_energy(Ko[a], Dm)
            assert abs(Ex[a, c] - Eo) < TOL_E * abs(Eo)


def test_two_kernels_equal_one_kernel_builds_768(exx):
    """On the 768-atom box each K^a equals build_K with V^a bit for bit, and so
    does each E_x; with V2 = V both results are identical."""
    sysm = synth.config(2)
    print("two kernels 768 atoms", flush=True)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    V2 = synth.short_range_V(inp)
    K2, Ex = two_build(plan, inp, V2)
    for a, Vx in enumerate((inp.V, V2)):
        K1, E1 = one_build(plan, inp, Vx)
        assert np.array_equal(K2[a], K1)
        assert np.array_equal(Ex[a], E1)
    Ks, _ = two_build(plan, inp, inp.V)
    assert np.array_equal(Ks[0], Ks[1])


def test_two_kernels_mixed_and_fp32(exx):
    """Mixed and all-FP32 two-kernel builds on the 768-atom box: each K^a equals
    build_K with V^a in the same precision bit for bit, and the mixed results
    are within the mixed bar of the FP64 two-kernel results."""
    sysm = synth.config(2)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    V2 = synth.short_range_V(inp)
    K64, E64 = two_build(plan, inp, V2)
    for prec in (exx.PREC_MIXED, exx.PREC_FP32):
        K2, Ex = two_build(plan, inp, V2, prec)
        for a, Vx in enumerate((inp.V, V2)):
            K1, E1 = one_build(plan, inp, Vx, prec)
            assert np.array_equal(K2[a], K1) and np.array_equal(Ex[a], E1)
        if prec == exx.PREC_MIXED:
            for a in range(2):
                dK, dE = np.abs(K2[a] - K64[a]).max(), abs(Ex[a, 0] - E64[a, 0]) / sysm.n_atoms
                print(f"mixed, kernel {a}: max|dK| {dK:.2e}, |dE|/atom {dE:.2e}", flush=True)
                assert dK <= 1e-5 and dE <= 1e-6
