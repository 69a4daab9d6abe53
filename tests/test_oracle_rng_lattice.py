"""Pins of the oracle's random numbers and Gauss-Hermite lattices (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(h, 16) for h in v["ctr"]]
        key = [int(h, 16) for h in v["key"]]
        out = [int(h, 16) for h in v["out"]]
        assert list(O.philox(ctr, key)) == out


def test_u53_edges():
    assert O.u53(0, 0) == 0.0
    assert O.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert O.u53(0x80000000, 0) == 0.5
    # the low word contributes only its top 21 bits
    assert O.u53(0, 0x7FF) == 0.0
    assert O.u53(0, 0x800) == 2.0 ** -53


def test_box_muller_closed_form():
    # -2 ln(1 - r1) = 1 gives radius 1; r2 = 1/8 gives angle pi/4
    z = O.box_muller(1.0 - math.exp(-0.5), 0.125)
    assert z == pytest.approx([math.sqrt(0.5), math.sqrt(0.5)], abs=1e-15)
    z = O.box_muller(0.0, 0.0)
    assert z[0] == 0.0 and z[1] == 0.0


def test_box_muller_statistics():
    # 2 * 20000 normals from a Philox stream: mean, variance, kurtosis within SE
    zs = []
    for i in range(20000):
        w = O.philox([i, 7, 0, 0], [1, 0])
        zs.extend(O.box_muller(O.u53(w[0], w[1]), O.u53(w[2], w[3])))
    z = np.array(zs)
    n = z.size
    assert abs(z.mean()) < 4.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert abs((z ** 4).mean() - 3.0) < 4.0 * math.sqrt(96.0 / n)


def _gauss_moment(p, q):
    return O._dfact(p) * O._dfact(q)


@pytest.mark.parametrize("Q,deg", [(9, 5), (37, 9)])
def test_lattice_gauss_hermite_exactness(Q, deg):
    lat = O.lattice(Q)
    xi, w = lat["xi"], lat["w"]
    assert np.all(w > 0) and abs(w.sum() - 1.0) < 1e-14
    for p in range(deg + 1):
        for q in range(deg + 1 - p):
            m = float(np.sum(w * xi[:, 0] ** p * xi[:, 1] ** q))
            assert m == pytest.approx(_gauss_moment(p, q), abs=1e-13 * max(1.0, _gauss_moment(p, q)))
    # one degree higher is no longer exact: the lattice is not accidentally better
    bad = max(abs(float(np.sum(w * xi[:, 0] ** p * xi[:, 1] ** (deg + 1 - p))) - _gauss_moment(p, deg + 1 - p))
              for p in range(deg + 2))
    assert bad > 1e-3


def test_d2q9_cannot_carry_xxx():
    # H_xxx and H_yyy vanish on every D2Q9 node, so D2Q9 keeps only a_xxy, a_xyy
    xi = O.lattice(9)["xi"]
    assert np.allclose(xi[:, 0] ** 3 - 3 * xi[:, 0], 0.0, atol=1e-14)
    assert np.allclose(xi[:, 1] ** 3 - 3 * xi[:, 1], 0.0, atol=1e-14)


def _hermite_basis(x, y, Q):
    """Orthogonal tensor components up to order 3 with their alpha! norms."""
    H = [(np.ones_like(x), 1.0), (x, 1.0), (y, 1.0),
         (x * x - 1, 2.0), (x * y, 1.0), (y * y - 1, 2.0),
         (x * x * y - y, 2.0), (x * y * y - x, 2.0)]
    if Q != 9:
        H += [(x ** 3 - 3 * x, 6.0), (y ** 3 - 3 * y, 6.0)]
    return H


@pytest.mark.parametrize("Q", [9, 37])
def test_lattice_hermite_orthogonality(Q):
    lat = O.lattice(Q)
    x, y, w = lat["xi"][:, 0], lat["xi"][:, 1], lat["w"]
    H = _hermite_basis(x, y, Q)
    for i, (hi, ni) in enumerate(H):
        for j, (hj, _) in enumerate(H):
            v = float(np.sum(w * hi * hj))
            assert v == pytest.approx(ni if i == j else 0.0, abs=1e-13)


def test_lattice_ordering_shells():
    e9 = O.lattice(9)["e"]
    e37 = O.lattice(37)["e"]
    assert np.array_equal(e37[:9], e9)
    assert len({tuple(v) for v in e37}) == 37
    assert np.array_equal(e37.sum(axis=0), [0, 0])
