"""Rejection sampler (Sec. III-B): the product's host logic against the oracle's
independent implementation on the same candidate / uniform streams (CPU only)."""
import numpy as np

import oracle
from paper_2110_09894_amd.sampling import rejection_sample
from workloads import random_grid_circuit, sampling_inputs


def test_sampler_matches_oracle_on_exact_amplitudes():
    circ = random_grid_circuit(3, 3, 6, 61)
    psi = oracle.statevector(circ)
    amps = np.transpose(psi, list(range(8, -1, -1))).reshape(-1)
    probs = oracle.probabilities(circ)
    assert np.allclose(np.abs(amps) ** 2, probs)
    cand, u = sampling_inputs(9, 4000, 5)
    got, info = rejection_sample(lambda c: amps[c.astype(np.int64)], 9, cand, u, 300, warmup=50, batch=97)
    want, dec = oracle.empirical_supremum_sample(probs, 9, cand, u, 300, warmup=50)
    assert np.array_equal(got, want)
    assert np.array_equal(info["decisions"], dec[:len(info["decisions"])])
    assert len(got) == 300


def test_sampler_distribution_close_to_exact():
    # with enough samples the empirical distribution approaches p (total variation)
    circ = random_grid_circuit(2, 3, 5, 62)
    probs = oracle.probabilities(circ)
    amps = np.sqrt(probs)  # only |a|^2 matters to the sampler
    cand, u = sampling_inputs(6, 200000, 9)
    got, _ = rejection_sample(lambda c: amps[c.astype(np.int64)], 6, cand, u, 20000, warmup=200, batch=4096)
    emp = np.bincount(got.astype(np.int64), minlength=64) / len(got)
    assert 0.5 * np.abs(emp - probs).sum() < 0.03


def test_warmup_samples_discarded_and_bound_grows():
    probs = np.full(16, 1 / 16)
    probs[3] = 0.4
    probs /= probs.sum()
    cand, u = sampling_inputs(4, 500, 3)
    got, info = rejection_sample(lambda c: np.sqrt(probs[c.astype(np.int64)]), 4, cand, u, 50, warmup=20)
    assert np.all(info["decisions"][:20] == -1)
    assert info["M"] >= probs.max() * 16 - 1e-12 or 3 not in cand[:info["candidates_used"]]


def _group_amps(amps, open_q):
    """Exact amplitudes of every candidate's group: [len, 2^m], member j has open qubit q_i = bit i of j."""
    qs = sorted(open_q)
    mask = sum(1 << q for q in qs)

    def fn(cand):
        out = np.empty((len(cand), 1 << len(qs)), dtype=np.complex128)
        for r, x in enumerate(cand):
            for j in range(1 << len(qs)):
                y = int(x) & ~mask
                for i, q in enumerate(qs):
                    y |= ((j >> i) & 1) << q
                out[r, j] = amps[y]
        return out
    return fn


def test_group_sampler_matches_oracle_on_exact_amplitudes():
    from paper_2110_09894_amd.sampling import rejection_sample_groups
    from workloads import group_sampling_inputs
    circ = random_grid_circuit(3, 3, 6, 63)
    psi = oracle.statevector(circ)
    amps = np.transpose(psi, list(range(8, -1, -1))).reshape(-1)
    probs = oracle.probabilities(circ)
    cand, u, c = group_sampling_inputs(9, 3000, 21)
    for open_q in ((4,), (0, 5, 7)):
        got, info = rejection_sample_groups(_group_amps(amps, open_q), 9, open_q, cand, u, c, 250, warmup=40,
                                            batch=61)
        want, dec = oracle.empirical_supremum_sample_groups(probs, 9, open_q, cand, u, c, 250, warmup=40)
        assert np.array_equal(got, want)
        assert np.array_equal(info["decisions"], dec[:len(info["decisions"])])
        assert len(got) == 250


def test_group_sampler_distribution_and_acceptance():
    # exact in distribution (total variation against p), and groups are accepted more often than single
    # bitstrings: their probabilities vary less, so the bound M is closer to the typical ratio
    from paper_2110_09894_amd.sampling import rejection_sample_groups
    from workloads import group_sampling_inputs
    circ = random_grid_circuit(2, 3, 5, 64)
    probs = oracle.probabilities(circ)
    amps = np.sqrt(probs)
    cand, u, c = group_sampling_inputs(6, 100000, 23)
    got, info = rejection_sample_groups(_group_amps(amps, (1, 4)), 6, (1, 4), cand, u, c, 20000, warmup=200,
                                        batch=4096)
    emp = np.bincount(got.astype(np.int64), minlength=64) / len(got)
    assert 0.5 * np.abs(emp - probs).sum() < 0.03
    single, sinfo = rejection_sample(lambda x: amps[x.astype(np.int64)], 6, cand, u, 20000, warmup=200,
                                     batch=4096)
    assert info["candidates_used"] < sinfo["candidates_used"]


def test_oracle_group_sampler_is_exact_in_distribution():
    # pins the oracle's group sampler to the definition: its samples follow p (total variation)
    from workloads import group_sampling_inputs
    circ = random_grid_circuit(2, 3, 5, 65)
    probs = oracle.probabilities(circ)
    cand, u, c = group_sampling_inputs(6, 60000, 25)
    got, dec = oracle.empirical_supremum_sample_groups(probs, 6, (0, 2, 5), cand, u, c, 12000, warmup=200)
    emp = np.bincount(got.astype(np.int64), minlength=64) / len(got)
    assert 0.5 * np.abs(emp - probs).sum() < 0.04
    assert np.all(dec[:200] == -1)
