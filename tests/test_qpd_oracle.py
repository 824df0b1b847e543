"""Pins of the QPD-sampling oracle (Sec. 4.3) against facts it must obey.

* Unbiasedness, exactly: the expectation of the sampled-and-truncated
  network's value over every multinomial outcome of the draws (enumerated
  with their probabilities) equals the exact contraction.  A wrong weight
  (dropped gamma, sign or 1/s_QPD), a truncation along the wrong axis or a
  kept index lost would all move it.
* Inverse-CDF draws: evenly spaced uniforms give every index within one
  draw of s_QPD |c_i| / gamma; zero coefficients are never drawn; a draw
  at the top of [0, 1) lands on the last non-zero index.
* A CT with one non-zero coefficient reduces to fixing its index (slicing).
* Large s_QPD: the estimate approaches the exact value within the bound
  the estimator's variance gives.
"""

import itertools
import math

import numpy as np
import pytest

from oracle import qpd_sampling as qs
from workloads import configs, qpd
from workloads.network import Network


def _einsum(net: Network) -> float:
    letters = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"
    spec = ",".join("".join(letters[l] for l in ls) for ls in net.labels) + "->"
    return float(np.einsum(spec, *[np.asarray(t, np.float64) for t in net.tensors], optimize=True))


def _triangle(seed: int) -> Network:
    # three QTs in a ring: two CZ gate cuts (dim 6) and one wire cut (dim 4)
    rng = np.random.default_rng(seed)
    dims = [6, 6, 4]
    labels = [[0, 2], [0, 1], [1, 2], [0], [1], [2]]
    tensors = [rng.uniform(-1, 1, (dims[ls[0]], dims[ls[1]])) for ls in labels[:3]]
    tensors += [qpd.CZ_COEFFS.copy(), qpd.CZ_COEFFS.copy(), qpd.WIRE_PAULI.copy()]
    return Network(tensors, labels, dims, [], ["qt"] * 3 + ["ct"] * 3)


def _compositions(s: int, k: int):
    for bars in itertools.combinations(range(s + k - 1), k - 1):
        prev, out = -1, []
        for b in bars + (s + k - 1,):
            out.append(b - prev - 1)
            prev = b
        yield np.array(out, dtype=np.int64)


def _pmf(counts, p) -> float:
    s = int(counts.sum())
    v = math.factorial(s)
    for n, q in zip(counts, p):
        v = v / math.factorial(int(n)) * q ** int(n)
    return v


@pytest.mark.parametrize("s_qpd", [1, 3])
def test_expectation_over_all_outcomes_is_exact(s_qpd):
    net = _triangle(5)
    exact = _einsum(net)
    p = np.abs(qpd.CZ_COEFFS) / np.abs(qpd.CZ_COEFFS).sum()
    outcomes = list(_compositions(s_qpd, 6))
    assert abs(sum(_pmf(o, p) for o in outcomes) - 1.0) < 1e-12
    expect = 0.0
    for n3 in outcomes:
        for n4 in outcomes:
            t = qs.truncate(net, [3, 4], [n3, n4], s_qpd)
            expect += _pmf(n3, p) * _pmf(n4, p) * _einsum(t)
    assert abs(expect - exact) <= 1e-12 * max(1.0, abs(exact))


def test_truncated_shapes_follow_the_counts():
    net = _triangle(1)
    n3 = np.array([2, 0, 1, 0, 0, 1])
    n4 = np.array([0, 0, 0, 4, 0, 0])
    t = qs.truncate(net, [3, 4], [n3, n4], 4)
    assert t.dims == [3, 1, 4]
    assert t.tensors[0].shape == (3, 4) and t.tensors[1].shape == (3, 1) and t.tensors[2].shape == (1, 4)
    # the wire CT is untouched; sampled CTs hold n_i gamma sign(c_i) / s
    assert np.array_equal(t.tensors[5], qpd.WIRE_PAULI)
    assert np.allclose(t.tensors[3], [1.5, 0.75, -0.75], rtol=0, atol=1e-15)
    assert np.allclose(t.tensors[4], [-3.0])
    # slices kept in index order
    assert np.array_equal(t.tensors[0], net.tensors[0][[0, 2, 5], :])
    assert np.array_equal(t.tensors[1], net.tensors[1][[0, 2, 5]][:, [3]])


def test_even_uniforms_track_the_probabilities():
    c = np.array([0.5, -0.25, 0.0, 1.25, -0.5, 0.5])
    p = np.abs(c) / np.abs(c).sum()
    for s in (1, 7, 64, 1000):
        u = (np.arange(s) + 0.5) / s
        n = qs.sample_counts(c, s, u)
        assert n.sum() == s
        assert n[2] == 0
        assert np.all(np.abs(n - s * p) <= 1.0)


def test_random_draws_match_the_distribution():
    c = qpd.CZ_COEFFS
    p = np.abs(c) / np.abs(c).sum()
    s = 60000
    u = np.random.default_rng(3).random(s)
    n = qs.sample_counts(c, s, u)
    sigma = np.sqrt(s * p * (1 - p))
    assert np.all(np.abs(n - s * p) < 5 * sigma)


def test_top_of_the_unit_interval_goes_to_the_last_nonzero_index():
    c = np.array([0.1, 0.7, 0.2, 0.0, 0.0])
    n = qs.sample_counts(c, 2, np.array([np.nextafter(1.0, 0.0), 0.0]))
    assert list(n) == [1, 0, 1, 0, 0]


def test_single_nonzero_coefficient_is_slicing():
    net = _triangle(2)
    net.tensors[3] = np.array([0.0, 0.0, -0.7, 0.0, 0.0, 0.0])
    n3 = qs.sample_counts(net.tensors[3], 5, np.random.default_rng(0).random(5))
    assert list(n3) == [0, 0, 5, 0, 0, 0]
    t = qs.truncate(net, [3], [n3], 5)
    assert t.tensors[3].shape == (1,) and abs(t.tensors[3][0] + 0.7) < 1e-15
    a, b, w = net.tensors[0][2], net.tensors[1][2], net.tensors[5]
    sliced = -0.7 * float(np.einsum("c,b,bc,b,c->", a, b, net.tensors[2], net.tensors[4], w))
    assert abs(_einsum(t) - sliced) < 1e-14


def test_grid_estimate_converges():
    # the mean of 40 independent sampled estimates of a 2x2 grid lies
    # within 5 standard errors of the exact value
    net = configs.grid_network(11, rows=2, cols=2)
    exact = _einsum(net)
    gate = [i for i, t in enumerate(net.tensors) if net.kinds[i] == "ct" and t.size == 6]
    assert gate
    rng = np.random.default_rng(4)
    s = 200
    vals = []
    for _ in range(40):
        cnts = [qs.sample_counts(net.tensors[c], s, rng.random(s)) for c in gate]
        vals.append(_einsum(qs.truncate(net, gate, cnts, s)))
    vals = np.array(vals)
    assert abs(vals.mean() - exact) < 5 * vals.std(ddof=1) / np.sqrt(len(vals)) + 1e-12


# --------------------------------------------------------------------------
# Fusion of the CTs between the same tensors before sampling (Sec. 4.3,
# Sec. 6.1 Step 1)
# --------------------------------------------------------------------------

def _double_bond(seed: int) -> Network:
    """QTs A[g0, g1, w] and B[w, g1, x, g0] joined by two CZ gate cuts
    (labels 0, 1: dim 6) and one wire cut (label 2: dim 4); B also meets C
    over a third gate cut (label 3).  The parallel gate cuts are listed out
    of label order in B, so the mode merge has to permute."""
    rng = np.random.default_rng(seed)
    dims = [6, 6, 4, 6]
    labels = [[0, 1, 2], [2, 1, 3, 0], [3], [0], [1], [2], [3]]
    tensors = [rng.uniform(-1, 1, [dims[l] for l in ls]) for ls in labels[:3]]
    tensors += [qpd.CZ_COEFFS.copy(), qpd.CZ_COEFFS.copy(), qpd.WIRE_PAULI.copy(), qpd.CZ_COEFFS.copy()]
    return Network(tensors, labels, dims, [], ["qt"] * 3 + ["ct"] * 4)


def test_parallel_groups_pair_the_cts_between_the_same_tensors():
    net = _double_bond(0)
    assert qs.parallel_groups(net, [3, 4, 6]) == [[3, 4], [6]]


def test_fusion_leaves_the_value_unchanged():
    # the fused network is an equivalent form: same contraction value, on a
    # hand-made double bond (modes out of order) and on ring-of-rings
    # networks with bond multiplicities 1-3
    import oracle
    for seed in range(4):
        net = _double_bond(seed)
        f, fids = qs.fuse_parallel(net, qs.parallel_groups(net, [3, 4, 6]))
        assert f.dims[0] == 36 and f.dims[1] == 1 and len(f.tensors) == len(net.tensors) - 1
        assert f.labels[1] == [2, 0, 3]      # B's two gate modes merged where the first of them stood
        assert abs(_einsum(f) - _einsum(net)) <= 1e-13 * max(1.0, abs(_einsum(net)))
    for seed in range(2):
        w = configs.ring_of_rings(seed)
        gate = [i for i, k in enumerate(w.kinds) if k == "ct" and w.tensors[i].size == 6]
        groups = qs.parallel_groups(w, gate)
        assert any(len(g) >= 2 for g in groups)
        f, _ = qs.fuse_parallel(w, groups)
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        fh, fl = oracle.ve_contract(f.tensors, f.labels, f.dims, f.out_labels)
        ref = float(hi) + float(lo)
        assert abs(float(fh) + float(fl) - ref) <= 1e-12 * abs(ref)


def test_fused_ct_is_the_tensor_product():
    # one-hot vectors fuse to the one-hot of the row-major pair index (first
    # CT slowest); k CZ cuts fuse to gamma = 3^k (the 9^k = gamma^(2k)
    # sampling overhead of Sec. 2.1) with coefficients still summing to 1
    dims = [6, 6, 6]
    e = [np.eye(6)[2], np.eye(6)[5], np.eye(6)[1]]
    labels = [[0, 1, 2], [0], [1], [2]]
    net = Network([np.zeros((6, 6, 6))] + e, labels, dims, [])
    f, fids = qs.fuse_parallel(net, [[1, 2, 3]])
    assert f.tensors[fids[0]].shape == (216,)
    assert np.flatnonzero(f.tensors[fids[0]]).tolist() == [2 * 36 + 5 * 6 + 1]
    for k in (1, 2, 3):
        net = Network([np.zeros((6,) * k)] + [qpd.CZ_COEFFS.copy() for _ in range(k)],
                      [list(range(k))] + [[i] for i in range(k)], [6] * k, [])
        f, fids = qs.fuse_parallel(net, [list(range(1, k + 1))])
        c = f.tensors[fids[0]]
        assert abs(np.abs(c).sum() - 3.0 ** k) < 1e-12 and abs(c.sum() - 1.0) < 1e-12


@pytest.mark.parametrize("s_qpd", [1, 2])
def test_fused_sampling_expectation_is_exact(s_qpd):
    # every multinomial outcome of the draws on the fused 36-entry CT and
    # on the single CT of the third cut, weighted by its probability
    net = _double_bond(7)
    exact = _einsum(net)
    groups = qs.parallel_groups(net, [3, 4, 6])
    f, fids = qs.fuse_parallel(net, groups)
    p0 = np.abs(f.tensors[fids[0]]) / np.abs(f.tensors[fids[0]]).sum()
    p1 = np.abs(f.tensors[fids[1]]) / np.abs(f.tensors[fids[1]]).sum()
    expect, total_p = 0.0, 0.0
    for n0 in _compositions(s_qpd, 36):
        for n1 in _compositions(s_qpd, 6):
            pr = _pmf(n0, p0) * _pmf(n1, p1)
            total_p += pr
            t = qs.truncate(f, fids, [n0, n1], s_qpd)
            # drawn pairs are kept jointly: at most s_QPD of the 36
            assert t.dims[0] <= s_qpd
            expect += pr * _einsum(t)
    assert abs(total_p - 1.0) < 1e-12
    assert abs(expect - exact) <= 1e-12 * max(1.0, abs(exact))


def test_simplify_keeps_drawn_pairs_of_the_original_modes():
    # one draw lands on pair (i, j) (and the third cut on k): the simplified
    # A is A[i, j, :] and B is B[:, j, k, i], with the fused CT's weight
    # gamma_f sign(c_i c_j), gamma_f = 9
    net = _double_bond(3)
    u = [np.array([0.5]), np.array([0.1])]
    simp, fused, fids, counts = qs.simplify(net, [3, 4, 6], 1, u)
    f = int(np.flatnonzero(counts[0])[0])
    k = int(np.flatnonzero(counts[1])[0])      # the third cut's drawn index
    i, j = divmod(f, 6)
    assert np.array_equal(simp.tensors[0].reshape(-1), net.tensors[0][i, j, :])
    assert np.array_equal(simp.tensors[1][:, 0, 0], net.tensors[1][:, j, k, i])
    c = qpd.CZ_COEFFS
    assert abs(simp.tensors[fids[0]][0] - 9.0 * np.sign(c[i] * c[j])) < 1e-15
