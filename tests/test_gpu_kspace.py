"""k-point Bloch sums of the real-space exchange matrix and density matrix,
and the strain derivative of the energy, through the C ABI, against the
oracle's Bloch sums and central differences of the oracle's energy."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import exx_oracle as O
from tests.gpu_util import device_inputs, relmax, run_build

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def exx():
    import paper_2403_10343_amd as m
    assert torch.cuda.is_available()
    return m


def _tiny(seed):
    lat = np.array([[3.0, 0.0, 0.0], [0.4, 3.2, 0.0], [0.2, -0.3, 3.4]])
    pos = np.array([[0.2, 0.3, 0.1], [2.6, 0.5, 0.4], [1.3, 2.9, 3.0], [1.5, 1.6, 1.7], [0.5, 2.8, 3.2]])
    return synth.System(np.array([0, 1, 1, 0, 1]), pos, 1.45, seed, lattice=lat)


GRID = np.array([(i / 3, j / 3, l / 3) for i in range(3) for j in range(3) for l in range(3)])


def _dk_from_real(inp, D, kpts, alias=True):
    """D(k) = sum_R e^{-i k.R} D(R) on the pair blocks, plus a term at a second image of
    one pair (which a full grid filters out)."""
    lay = inp.layout
    nb = inp.system.basis_table[inp.system.species].astype(np.int64)
    bo = np.concatenate([[0], np.cumsum(nb)])
    n = D.shape[0]
    q = next(p for p in range(lay.n_pairs) if lay.pair_a[p] != lay.pair_b[p])
    a, b = int(lay.pair_a[q]), int(lay.pair_b[q])
    Z = np.random.default_rng(0).normal(size=(nb[a], nb[b]))
    out = np.zeros((len(kpts), n, n), dtype=complex)
    for t, k in enumerate(kpts):
        for pa, pb, nn in zip(lay.pair_a, lay.pair_b, lay.pair_img):
            ia, ib = slice(bo[pa], bo[pa + 1]), slice(bo[pb], bo[pb + 1])
            ph = np.exp(-2j * np.pi * float(k @ nn))
            out[t, ia, ib] = ph * D[ia, ib]
            out[t, ib, ia] = np.conj(ph) * D[ib, ia]
        if alias:
            ia, ib = slice(bo[a], bo[a + 1]), slice(bo[b], bo[b + 1])
            ph = np.exp(-2j * np.pi * float(k @ (np.asarray(lay.pair_img[q]) + [1, 0, 0])))
            out[t, ia, ib] += ph * Z
            out[t, ib, ia] += np.conj(ph) * Z.T
    return out


@pytest.mark.parametrize("which", ["tiny", "cell"])
def test_bloch_sum_and_density_from_k(exx, which):
    """K(k) of the GPU's X against the oracle's Bloch sum; D(k) on a full 3x3x3
    grid back to the folded D (a second image of one pair filtered out); the
    build on that D equals the build on D; -1/4 (1/N_k) sum_k <K(k), D(k)>
    equals the GPU's E_x."""
    sysm = _tiny(3) if which == "tiny" else synth.ice_box_periodic(1, 1, 1, seed=4, r_cut=3.4)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    K, Ex = run_build(plan, inp, torch)
    n = int(inp.layout.sys_nbas[0])
    X = K.reshape(n, n)
    kpts = np.array([(0.25, -0.1, 0.4), (0.5, 0.5, 0.0), (-0.3, 0.2, 0.1), (0.0, 0.0, 0.0)])
    Kk = plan.bloch_sum(torch.from_numpy(K).to("cuda:0"), kpts).cpu().numpy()
    Ko = O.bloch_sum(inp, X, kpts)
    for t in range(len(kpts)):
        assert relmax(Kk[t].reshape(n, n), Ko[t]) < 1e-14
    assert np.array_equal(Kk[3].real, K) and not Kk[3].imag.any()
    D = inp.D.reshape(n, n)
    Dk = _dk_from_real(inp, D, GRID)
    Dg = plan.density_from_k(torch.from_numpy(Dk.reshape(len(GRID), -1)).to("cuda:0"), GRID).cpu().numpy()
    assert relmax(Dg.reshape(n, n), D) < 1e-13
    assert relmax(Dg.reshape(n, n), O.density_from_k(inp, list(Dk), GRID)) < 1e-13
    K2, E2 = run_build(plan, O.with_density(inp, Dg), torch)
    assert relmax(K2, K) < 1e-12 and abs(E2[0] - Ex[0]) < 1e-12 * abs(Ex[0])
    Kg = plan.bloch_sum(torch.from_numpy(K).to("cuda:0"), GRID).cpu().numpy()
    e_k = -0.25 * np.real(np.sum(Kg.reshape(len(GRID), n, n) * Dk)) / len(GRID)
    print(f"{which}: E_x {Ex[0]:.12e}, from k-space {e_k:.12e}", flush=True)
    assert abs(e_k - Ex[0]) < 1e-12 * abs(Ex[0])


def test_bloch_sum_cluster_and_errors(exx):
    sysm = synth.water_cluster(2, 3)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    K, _ = run_build(plan, inp, torch)
    Kk = plan.bloch_sum(torch.from_numpy(K).to("cuda:0"), [(0.3, 0.1, -0.2)]).cpu().numpy()
    assert np.array_equal(Kk[0].real, K) and not Kk[0].imag.any()   # a cluster has R = 0 only
    Xd = torch.from_numpy(K).to("cuda:0")
    with pytest.raises(exx.ExxError) as e:
        plan.bloch_sum(Xd, np.zeros((0, 3)))
    assert e.value.code == -1
    with pytest.raises(exx.ExxError) as e:
        plan.bloch_sum(Xd, [(float("nan"), 0.0, 0.0)])
    assert e.value.code == -1


def _strained(sysm, eps):
    F = np.eye(3) + eps
    kw = dict(pos=sysm.pos @ F.T)
    if sysm.lattice is not None:
        kw["lattice"] = sysm.lattice @ F.T
    return dataclasses.replace(sysm, **kw)


@pytest.mark.parametrize("which", ["cluster", "periodic"])
def test_strain_derivative_central_differences(exx, which):
    """dE/d(eps) from the GPU gradients against central differences (step 1e-4)
    of the oracle's E_x under x -> (1 + eps) x (positions and lattice; C and V
    regenerated, D and the pair lists held fixed); symmetric."""
    sysm = synth.water_cluster(2, 5) if which == "cluster" else _tiny(5)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    C, V, D = device_inputs(inp, torch)
    dC, dV = torch.empty_like(C), torch.empty_like(V)
    plan.exchange_backward(C, V, D, 1.0, dC=dC, dV=dV)
    W = plan.strain_derivative(C, V, dC, dV).cpu().numpy()
    n = int(inp.layout.sys_nbas[0])

    def energy(eps):
        i2 = synth.make_inputs(_strained(sysm, eps), inp.layout)
        i2.D[:] = inp.D
        if which == "cluster":
            return O.exchange_energy(O.k_eigen(i2), i2.D.reshape(n, n))
        return O.periodic_energy(O.x_periodic(i2), i2.D.reshape(n, n))

    h = 1e-4
    fd = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            fd[a, b] = (energy(e) - energy(-e)) / (2 * h)
    print(f"{which}: dE/deps\n{W}\nFD\n{fd}", flush=True)
    assert np.abs(W - fd).max() < 1e-6 * np.abs(fd).max()
    assert np.abs(W - W.T).max() < 1e-12 * np.abs(W).max()


def test_strain_derivative_768_box_spin(exx):
    """768-atom box: symmetric; the spin gradients with equal spins D/2 give
    the one-density strain derivative."""
    sysm = synth.config(2)
    inp = synth.make_inputs(sysm)
    plan = exx.Plan.for_system(sysm)
    C, V, D = device_inputs(inp, torch)
    dC, dV = torch.empty_like(C), torch.empty_like(V)
    plan.exchange_backward(C, V, D, 1.0, dC=dC, dV=dV)
    W = plan.strain_derivative(C, V, dC, dV).cpu().numpy()
    D2 = torch.cat([0.5 * D, 0.5 * D])
    plan.exchange_backward_spin(C, V, D2, 1.0, dC=dC, dV=dV)
    Ws = plan.strain_derivative(C, V, dC, dV).cpu().numpy()
    assert np.abs(W - W.T).max() < 1e-12 * np.abs(W).max()
    assert np.abs(Ws - W).max() < 1e-12 * np.abs(W).max()
