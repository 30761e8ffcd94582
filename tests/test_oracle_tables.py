"""Pins of the oracle's lattice tables against Table I and the moment
conditions of Sec. II (Eqs. (3)-(4)) and Sec. III (Eq. (17))."""
from fractions import Fraction

import pytest

import oracle
from conftest import read_golden


def _exact(x: float, q: Fraction) -> bool:
    # the double must be the correctly rounded value of the rational
    return float(q) == x


@pytest.fixture(scope="module")
def tab():
    return oracle.tables()


def _classes(tab):
    return [ex * ex + ey * ey for ex, ey in zip(tab["ex"], tab["ey"])]


def test_weights_match_table1(tab):
    cls = _classes(tab)
    for row in read_golden("table1_weights.txt"):
        kind, c, count, num, den = row.split()
        c, count, q = int(c), int(count), Fraction(int(num), int(den))
        key = "p" if kind == "p" else "w"
        members = [i for i in range(25) if cls[i] == c]
        assert len(members) == count, (kind, c)
        for i in members:
            assert _exact(tab[key][i], q), (kind, i, tab[key][i], q)
    # w vanishes on the second belt
    assert all(tab["w"][i] == 0.0 for i in range(25) if cls[i] > 2)


def test_speed_sets_distinct_and_symmetric(tab):
    vecs = list(zip(tab["ex"], tab["ey"]))
    assert len(set(vecs)) == 25 and vecs[0] == (0, 0)
    for v in vecs:
        assert (-v[0], -v[1]) in vecs
    assert all(max(abs(a), abs(b)) == 1 for a, b in vecs[1:9])
    assert all(max(abs(a), abs(b)) == 2 for a, b in vecs[9:])
    # the first belt is the D2Q9 kinetic set, same order
    assert vecs[1:9] == list(zip(tab["cx"], tab["cy"]))[1:9]


def _moment(tab, key, fx):
    return sum(Fraction(tab[key][i]).limit_denominator(20000) * fx(tab["ex"][i], tab["ey"][i])
               for i in range(25))


def test_normalisation_and_sound_speed(tab):
    # Eq. (3): both weight sets sum to one; Eq. (4): second moments = c_s^2 = 1/3
    assert _moment(tab, "p", lambda x, y: 1) == 1
    assert _moment(tab, "w", lambda x, y: 1) == 1
    for key in ("p", "w"):
        assert _moment(tab, key, lambda x, y: x * x) == Fraction(1, 3)
        assert _moment(tab, key, lambda x, y: y * y) == Fraction(1, 3)
        assert _moment(tab, key, lambda x, y: x * y) == 0


def test_isotropy_orders(tab):
    # Sec. II: 4th-order isotropy on belt 1 (w), 8th order with both belts (p).
    # Isotropic tensors need sum c_x^4 = 3 sum c_x^2 c_y^2, sum c_x^6 = 5 sum c_x^4 c_y^2,
    # sum c_x^8 = 7 sum c_x^6 c_y^2 = (35/3) sum c_x^4 c_y^4.
    m = lambda key, a, b: _moment(tab, key, lambda x, y: x ** a * y ** b)
    assert m("w", 4, 0) == 3 * m("w", 2, 2)
    assert m("p", 4, 0) == 3 * m("p", 2, 2)
    assert m("p", 6, 0) == 5 * m("p", 4, 2)
    assert m("p", 8, 0) == 7 * m("p", 6, 2)
    assert m("p", 8, 0) == Fraction(35, 3) * m("p", 4, 4)
    # odd moments vanish
    assert m("p", 1, 0) == 0 and m("p", 3, 0) == 0 and m("p", 2, 1) == 0


def test_effective_coupling_ratio(tab):
    # Eq. (17): G_s2 = G^a + (12/7) G^r is the ratio of the fourth moments of
    # the p and w sets; G_s1 = G^a + G^r is the ratio of the second moments.
    m = lambda key, a, b: _moment(tab, key, lambda x, y: x ** a * y ** b)
    assert m("p", 2, 2) / m("w", 2, 2) == Fraction(12, 7)
    assert m("p", 4, 0) / m("w", 4, 0) == Fraction(12, 7)
    assert m("p", 2, 0) / m("w", 2, 0) == 1


def test_d2q9_set(tab):
    # D2Q9 weights (Table I, w) and c_s^2 = 1/3; the kinetic set's fourth moments
    # give the isotropic second-order equilibrium.
    w = [Fraction(v).limit_denominator(100) for v in tab["wq"]]
    cx, cy = tab["cx"], tab["cy"]
    assert sum(w) == 1
    assert sum(wi * x * x for wi, x in zip(w, cx)) == Fraction(1, 3)
    assert sum(wi * x ** 4 for wi, x in zip(w, cx)) == 3 * sum(wi * x * x * y * y for wi, x, y in zip(w, cx, cy))
    assert w[0] == Fraction(4, 9)
