"""Pins of the oracle's pair integrals over a range [a, b) (Section 2.2):
closed forms, the single-PCF oracle (segment iteration) against the zero
PCF, additivity over the bounds, and the restriction identity
int_a^b h(f, g) = int_0^inf h(f 1_[a,b), g 1_[a,b)) (h(0, 0) = 0 for every
kind) with the restriction written out here in NumPy."""
import math

import numpy as np
import pytest

import oracle
from paper_2404_07183_amd import workloads

INF = math.inf


def _set(*pcfs):
    o = np.concatenate([[0], np.cumsum([len(t) for t, _ in pcfs])])
    return (o, np.concatenate([np.asarray(t, float) for t, _ in pcfs]),
            np.concatenate([np.asarray(v, float) for _, v in pcfs]))


def restrict(t, v, a, b):
    """Rows of f * 1_[a, b) for one PCF (t, v) (plain NumPy)."""
    k = np.searchsorted(t, a, side="right") - 1
    rows_t, rows_v = ([0.0, a], [0.0, v[k]]) if a > 0 else ([0.0], [v[0]])
    inside = (t > a) & (t < b)
    rows_t += list(t[inside])
    rows_v += list(v[inside])
    if b < INF:
        rows_t.append(b)
        rows_v.append(0.0)
    return np.array(rows_t), np.array(rows_v)


def test_closed_forms():
    o, t, v = _set(([0.0, 1.0, 4.0], [2.0, -3.0, 0.0]), ([0.0, 2.0], [1.0, 0.0]))
    E = lambda kind, p, a, b: oracle.entries_ab(kind, p, a, b, o, t, v, [0], [1])[0]
    assert E(oracle.LP, 1.0, 0.5, 3.0) == 0.5 * 1 + 1 * 4 + 1 * 3
    assert E(oracle.GRAM, 0.0, 0.5, 3.0) == 2 * 0.5 - 3 * 1
    assert E(oracle.LP_POW, 2.0, 0.5, 3.0) == 0.5 * 1 + 1 * 16 + 1 * 9
    assert E(oracle.LP, 1.0, 5.0, 7.0) == 0.0
    assert E(oracle.LP, 1.0, 0.0, INF) == oracle.entries(oracle.LP, 1.0, o, t, v, [0], [1])[0]
    with pytest.raises(ValueError):
        oracle.entries_ab(oracle.LP, 1.0, 3.0, 3.0, o, t, v, [0], [1])


@pytest.mark.parametrize("seed", [1, 2])
def test_against_single_functionals(seed):
    # d_p(f, 0)^p over [a, b) = int_a^b |f|^p by segment iteration
    o, t, v = workloads.uniform_counts(25, 1, 60, seed=seed)
    o2 = np.concatenate([o, [o[-1] + 1]])
    t2, v2 = np.concatenate([t, [0.0]]), np.concatenate([v, [0.0]])  # + the zero PCF
    n = len(o) - 1
    rng = np.random.default_rng(seed)
    for a, b in [(0.0, INF), (0.0, 10.0), tuple(np.sort(rng.uniform(0, 40, 2))), (7.0, INF)]:
        for p in (1.0, 2.0, 3.5):
            got, ab = oracle.entries_ab(oracle.LP_POW, p, a, b, o2, t2, v2, np.arange(n),
                                        np.full(n, n), with_abs=True)
            ref = oracle.single(oracle.S_NORM_POW, p, a, b, o, t, v)
            assert np.all(np.abs(got - ref) <= 1e-13 * ab + 1e-300), (a, b, p)


@pytest.mark.parametrize("seed", [3, 4])
def test_additivity_and_restriction(seed):
    o, t, v = workloads.uniform_counts(20, 1, 50, seed=seed)
    rng = np.random.default_rng(seed)
    I = rng.integers(0, 20, 30)
    J = rng.integers(0, 20, 30)
    for _ in range(4):
        a, c, b = np.sort(rng.uniform(0, 45, 3))
        for kind, p in ((oracle.LP_POW, 2.0), (oracle.GRAM, 0.0), (oracle.LP_POW, 1.0)):
            x, s1 = oracle.entries_ab(kind, p, a, c, o, t, v, I, J, with_abs=True)
            y, s2 = oracle.entries_ab(kind, p, c, b, o, t, v, I, J, with_abs=True)
            z = oracle.entries_ab(kind, p, a, b, o, t, v, I, J)
            assert np.all(np.abs(x + y - z) <= 1e-12 * (s1 + s2) + 1e-300)
            # the restricted PCFs over [0, inf) give the same integrals
            rows = [restrict(t[o[i]:o[i + 1]], v[o[i]:o[i + 1]], a, b) for i in range(20)]
            ro, rt, rv = _set(*rows)
            w, sw = oracle.entries(kind, p, ro, rt, rv, I, J, with_abs=True)
            assert np.all(np.abs(w - z) <= 1e-12 * sw + 1e-300)
