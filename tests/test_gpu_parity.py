"""FP64 GPU path against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest

import synth
from oracle import exx_oracle as O
from tests.gpu_util import relmax, run_build, system_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_K = 1e-10          # max|dK| / max|K|, FP64 path
TOL_E = 1e-10          # relative, E_x


@pytest.fixture(scope="module")
def exx():
    import paper_2403_10343_amd as m
    assert torch.cuda.is_available()
    return m


def _plan(exx, sysm):
    return exx.Plan.for_system(sysm)


def test_device_screening_matches_layout(exx):
    for sysm in (synth.config(1), synth.cluster_batch(5, n_min=8, n_max=40), synth.config(2)):
        print("screening", sysm.name, flush=True)
        lay = synth.make_layout(sysm)
        p = _plan(exx, sysm)
        pa, pb, co, vo = p.pairs()
        assert np.array_equal(pa, lay.pair_a) and np.array_equal(pb, lay.pair_b)
        assert np.array_equal(co, lay.c_off) and np.array_equal(vo, lay.v_off)
        hp = exx.Plan.for_system(sysm, host_only=True)
        for x, y in zip(p.neighbors(), hp.neighbors()):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("n_mol", [1, 2, 3, 8])
def test_K_fp64_cluster(exx, n_mol):
    sysm = synth.water_cluster(n_mol, seed=n_mol)
    print("cluster", n_mol, flush=True)
    inp = synth.make_inputs(sysm)
    K, Ex = run_build(_plan(exx, sysm), inp, torch)
    Kg = system_block(K, inp.layout, 0)
    Ko = O.k_eigen(inp)
    assert relmax(Kg, Ko) < TOL_K
    Eo = O.exchange_energy(Ko, O.Blocks(inp).D)
    assert abs(Ex[0] - Eo) < TOL_E * abs(Eo)
    assert np.array_equal(Kg, Kg.T)


def test_K_fp64_config1_4index(exx):
    """Config 1 (8 waters, 24 atoms) against the 4-index route; E_x also from (ij|kl)."""
    inp = synth.make_inputs(synth.config(1))
    K, Ex = run_build(_plan(exx, inp.system), inp, torch)
    K4, e_k, e_direct = O.k_4index(inp)
    assert relmax(system_block(K, inp.layout, 0), K4) < TOL_K
    assert abs(Ex[0] - e_direct) < TOL_E * abs(e_direct)


def test_single_atom_and_pair(exx):
    for species, pos in (([synth.O], [[0, 0, 0]]), ([synth.H], [[0, 0, 0]]),
                         ([synth.O, synth.H], [[0, 0, 0], [0, 0, 0.96]]),
                         ([synth.H, synth.H], [[0, 0, 0], [0, 0, 7.0]])):
        sysm = synth.System(np.array(species), np.array(pos, float), 6.0, seed=3)
        inp = synth.make_inputs(sysm)
        K, Ex = run_build(_plan(exx, sysm), inp, torch)
        assert relmax(system_block(K, inp.layout, 0), O.k_eigen(inp)) < TOL_K


def test_batch_of_uneven_clusters(exx):
    b = synth.cluster_batch(6, n_min=1, n_max=12)
    inp = synth.make_inputs(b)
    K, Ex = run_build(_plan(exx, b), inp, torch)
    for s in range(b.n_systems):
        Ko = O.k_eigen(inp, s)
        assert relmax(system_block(K, inp.layout, s), Ko) < TOL_K
        Eo = O.exchange_energy(Ko, O.Blocks(inp, s).D)
        assert abs(Ex[s] - Eo) < TOL_E * abs(Eo)


def test_zero_D_and_linearity_and_determinism(exx):
    sysm = synth.water_cluster(4, seed=9)
    inp = synth.make_inputs(sysm)
    plan = _plan(exx, sysm)
    K1, _ = run_build(plan, inp, torch)
    K1b, _ = run_build(plan, inp, torch)
    assert np.array_equal(K1, K1b), "run-to-run results differ"
    z = synth.Inputs(sysm, inp.layout, inp.C, inp.V, np.zeros_like(inp.D))
    K0, E0 = run_build(plan, z, torch)
    assert not np.any(K0) and E0[0] == 0.0
    inp2 = synth.make_inputs(synth.System(sysm.species, sysm.pos, sysm.r_cut, seed=99))
    mix = synth.Inputs(sysm, inp.layout, inp.C, inp.V, 0.3 * inp.D - 1.7 * inp2.D)
    K2, _ = run_build(plan, synth.Inputs(sysm, inp.layout, inp.C, inp.V, inp2.D), torch)
    Km, _ = run_build(plan, mix, torch)
    assert relmax(Km, 0.3 * K1 - 1.7 * K2) < 1e-12


def test_config2_sampled_rows(exx):
    """768-atom box at full size, in the benchmark's launch configuration (tile
    shapes chosen by the autotuner on these inputs): sampled rows of K against
    the row oracle, symmetry, and E_x from K."""
    from tests.gpu_util import device_inputs
    inp = synth.make_inputs(synth.config(2))
    plan = _plan(exx, inp.system)
    C, V, D = device_inputs(inp, torch)
    Kt = torch.empty(plan.info["d_size"], dtype=torch.float64, device="cuda:0")
    plan.autotune(C, V, D, Kt)
    print("tuned tile shapes", {k: v[0] for k, v in plan.tuning().items()}, flush=True)
    K, Ex = run_build(plan, inp, torch)
    Kg = system_block(K, inp.layout, 0)
    rng = np.random.default_rng(0)
    rows = np.concatenate([[0, 6143], rng.integers(0, 6144, 4)])
    blk = O.Blocks(inp)
    Kr = O.k_rows(inp, rows, blk=blk)
    scale = np.abs(Kg).max()
    assert np.abs(Kg[rows] - Kr).max() < TOL_K * scale
    assert np.array_equal(Kg, Kg.T)
    assert abs(Ex[0] - O.exchange_energy(Kg, blk.D)) < 1e-12 * abs(Ex[0])


def test_hand_worked_two_atom_case(exx):
    """Two one-function atoms; K and E_x worked out by hand (tests/golden)."""
    from tests.test_oracle import golden_inputs
    inp, g = golden_inputs("two_atom_hand.json")
    K, Ex = run_build(_plan(exx, inp.system), inp, torch)
    assert np.abs(K - np.array(g["K"])).max() < 1e-12
    assert abs(Ex[0] - g["E_x"]) < 1e-12


@pytest.mark.parametrize("tables", [([16, 3], [64, 7]), ([7, 1], [23, 2]), ([1, 2], [1, 5]),
                                    ([16, 16], [64, 64]), ([12, 9], [33, 17])])
def test_other_species_shapes(exx, tables):
    """Basis / aux counts away from the water species, up to the limits
    (16 basis, 64 aux per atom): every shape class of the kernels, ragged
    tiles, groups of up to 8 aux tiles."""
    nb, na = tables
    base = synth.water_cluster(4, seed=17)
    sysm = synth.System(base.species, base.pos, 6.0, seed=17,
                        basis_table=np.array(nb), aux_table=np.array(na))
    print("species tables", tables, flush=True)
    inp = synth.make_inputs(sysm)
    K, Ex = run_build(_plan(exx, sysm), inp, torch)
    Kg = system_block(K, inp.layout, 0)
    Ko = O.k_eigen(inp)
    assert relmax(Kg, Ko) < TOL_K
    Eo = O.exchange_energy(Ko, O.Blocks(inp).D)
    assert abs(Ex[0] - Eo) < TOL_E * abs(Eo)


def _row_sample(inp, n_atoms_each=3, rows_per_atom=4, seed=1):
    """Rows of K on O and H atoms at the surface (fewest neighbours) and in the
    interior (most neighbours) of a box: n_atoms_each atoms of each kind, the
    first, last and random basis rows of each."""
    blk = O.Blocks(inp)
    deg = np.array([len(x) for x in blk.nbrs])
    sp = inp.system.species
    rng = np.random.default_rng(seed)
    rows = []
    for s in (synth.O, synth.H):
        atoms = np.nonzero(sp == s)[0]
        order = atoms[np.argsort(deg[atoms], kind="stable")]
        for a in list(order[:n_atoms_each]) + list(order[-n_atoms_each:]):
            b0, nb = int(blk.bo[a]), int(blk.nb[a])
            pick = [b0, b0 + nb - 1] + list(b0 + rng.choice(np.arange(1, nb - 1), rows_per_atom - 2, replace=False))
            rows += pick
    return np.array(rows), blk


def test_config2_48_oracle_rows_fp64_and_mixed(exx):
    """48 rows of K of the 768-atom box (O and H rows of surface and interior
    atoms) against the oracle's row route: FP64 at 1e-10 relative, the mixed
    build (default split) at the 1e-5 absolute bar."""
    inp = synth.make_inputs(synth.config(2))
    plan = _plan(exx, inp.system)
    rows, blk = _row_sample(inp)
    assert len(rows) == 48 and len(set(rows.tolist())) == 48
    K, _ = run_build(plan, inp, torch)
    Km, _ = run_build(plan, inp, torch, exx.PREC_MIXED)
    print("oracle rows:", rows.tolist(), flush=True)
    Kr = O.k_rows(inp, rows, blk=blk)
    Kg = system_block(K, inp.layout, 0)[rows]
    Kmg = system_block(Km, inp.layout, 0)[rows]
    scale = np.abs(Kr).max()
    print(f"48 rows: fp64 rel {np.abs(Kg - Kr).max() / scale:.2e}, mixed abs {np.abs(Kmg - Kr).max():.2e}", flush=True)
    assert np.abs(Kg - Kr).max() < TOL_K * scale
    assert np.abs(Kmg - Kr).max() <= 1e-5
