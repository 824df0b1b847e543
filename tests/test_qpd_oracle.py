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
