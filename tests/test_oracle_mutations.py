"""Plant plausible mistakes in a copy of the oracle and check that at least
one pin catches each of them (the pins are strong enough to matter)."""
import os
import types

import pytest

from tests import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "exx_oracle.py")

MUTATIONS = {
    "no_mirror_of_C": ("C3[mu, ib, ia] = part.transpose(0, 2, 1)", "pass"),
    "swapped_aux_owner": ("for owner, part in ((a, blk[:self.na[a]]), (b, blk[self.na[a]:])):",
                          "for owner, part in ((b, blk[:self.na[a]]), (a, blk[self.na[a]:])):"),
    "V_not_mirrored": ("Vd[mb, ma] = blk.T", "pass"),
    "D_transposed_in_4index": ('K[i0:i1] = np.einsum("ijkl,jl->ik", eri, D, optimize=True)',
                               'K[i0:i1] = np.einsum("ijkl,lj->ik", eri, D, optimize=True)'),
    "energy_factor": ("return -0.25 * float(np.sum(K * D))", "return -0.5 * float(np.sum(K * D))"),
    "onsite_dV_factor": ("vg = -0.25 * tau[ma, ma]", "vg = -0.5 * tau[ma, ma]"),
    "offsite_dC_factor": ("g = np.concatenate([G[ma, ia, ib], G[mb, ia, ib]]) * 2.0",
                          "g = np.concatenate([G[ma, ia, ib], G[mb, ia, ib]])"),
    "force_V_sign": ("grads[\"sV\"][q] * (-2.0 / v_2s2) * d", "grads[\"sV\"][q] * (2.0 / v_2s2) * d"),
    "rows_wrong_orientation": ('Ki[sq] += np.einsum("nkl,nk->l", part, yQ[:, sj])',
                               'Ki[sq] += np.einsum("nkl,nl->k", part, yQ[:, sj])'),
    "rows_missing_transpose_term": ('Ki[sj] += np.einsum("nkl,nk->l", part, yQ[:, sq])', "pass"),
    "eigen_missing_lambda": ("Ul = U * lam[None, None, :]", "Ul = U"),
    "screening_strict": ("a, b = np.nonzero(np.triu(r2 <= rc2))", "a, b = np.nonzero(np.triu(r2 < 0.81 * rc2))"),
    "spin_energy_factor": ("return -0.5 * sum(float(np.sum(K * D))", "return -0.25 * sum(float(np.sum(K * D))"),
    "two_kernels_same_V": ("return [f(inputs, s), f(with_coulomb(inputs, V2), s)]",
                           "return [f(inputs, s), f(inputs, s)]"),
    "block_missing_mirror_term": ('KI[:, sj] += np.einsum("nkl,nik->il", part, yQ, optimize=True)', "pass"),
    "block_V_not_transposed": ("VPQ = vb if P <= Q else vb.T                   # [mu on P, nu on Q]",
                               "VPQ = vb if P <= Q else vb                     # [mu on P, nu on Q]"),
    "periodic_flip_image_sign": ("return [((J, m), blk[:self.na[J]].transpose(0, 2, 1)), ((I, (0, 0, 0)), blk[self.na[J]:].transpose(0, 2, 1))]",
                                 "return [((J, m), blk[self.na[J]:].transpose(0, 2, 1)), ((I, (0, 0, 0)), blk[:self.na[J]].transpose(0, 2, 1))]"),
    "periodic_D_any_image": ("ok = (tab[np.ix_(rj, cl)] >= 0) & (tab[np.ix_(rj, cl)] + rm[:, None] - code(zero) == cb[None, :])",
                             "ok = tab[np.ix_(rj, cl)] >= 0"),
    "periodic_V_relative_image": ("        r = tuple(b - a for a, b in zip(p, q))", "        r = q"),
    "spin_ignores_D": ("return [f(with_density(inputs, D), s) for D in D_spin]",
                       "return [f(inputs, s) for D in D_spin]"),
    "estimate_sigma_one_hop": ("        sigma[a] = max(sigma[a], rho[b])\n        sigma[b] = max(sigma[b], rho[a])",
                               "        sigma[a] = max(sigma[a], rho[a])\n        sigma[b] = max(sigma[b], rho[b])"),
    "estimate_tau_of_first_atom": ("            tau[x] = max(tau[x], norms[p, 0])",
                                   "            tau[a] = max(tau[a], norms[p, 0])"),
    "estimate_max_for_min": ("* min(sigma[a], sigma[b])", "* max(sigma[a], sigma[b]) * 0.5"),
    "norms_C_first_atom_only": ("out[p, 0] = np.abs(inputs.C[lay.c_off[p]:lay.c_off[p + 1]]).max()",
                                "out[p, 0] = np.abs(inputs.C[lay.c_off[p]:(lay.c_off[p] + lay.c_off[p + 1]) // 2]).max()"),
    "spin_gradient_factor": ("out = {k: 2.0 * (parts[0][k] + parts[1][k]) for k in", "out = {k: (parts[0][k] + parts[1][k]) for k in"),
    "spin_dD_one_density": ('out["dD"] = [2.0 * p["dD"] for p in parts]', 'out["dD"] = [p["dD"] for p in parts]'),
    "bloch_same_phase_both_blocks": ("            Kk[ib, ia] = np.conj(ph) * X[ib, ia]", "            Kk[ib, ia] = ph * X[ib, ia]"),
    "density_k_no_average": ("ph[q] * Dk[q][ia, ib] for q in range(len(kp)))) / len(kp)",
                             "ph[q] * Dk[q][ia, ib] for q in range(len(kp))))"),
    "density_k_phase_sign": ("        ph = np.exp(2j * np.pi * (kp @ nab))", "        ph = np.exp(-2j * np.pi * (kp @ nab))"),
    "screened_V_neighbour_block": ("        V[lay.v_off[p]:lay.v_off[p + 1]] = 0.0",
                                   "        V[lay.v_off[p]:lay.v_off[p + 1] - 1] = 0.0"),
}


def _mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique / missing: {old!r}"
    mod = types.ModuleType("exx_oracle_mutant")
    exec(compile(src.replace(old, new), "exx_oracle_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    mod = _mutant(*MUTATIONS[name])
    monkeypatch.setattr(pins, "O", mod)
    failed = []
    for pin_name, pin in pins.ALL_PINS.items():
        try:
            ok, _ = pin()
        except Exception:
            ok = False
        if not ok:
            failed.append(pin_name)
            break
    assert failed, f"mutation {name} was not caught by any pin"
