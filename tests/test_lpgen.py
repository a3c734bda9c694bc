"""The seeded input generator: Philox known answers, determinism, recipes."""
import os

import numpy as np

import lpgen

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [ln.split() for ln in open(GOLD) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(v, 16) for v in r]
        assert lpgen.philox4x32_10(w[0:4], w[4:6]) == w[6:10]


def test_deterministic_and_subset_independent():
    a = lpgen.config(2, range(0, 6))
    b = lpgen.config(2, [3, 5])
    la, lb = a.lp(3), b.lp(0)
    assert np.array_equal(la["A"], lb["A"]) and np.array_equal(la["b"], lb["b"])
    assert np.array_equal(a.lp(5)["c"], b.lp(1)["c"])
    c = lpgen.config(2, range(0, 6))
    assert np.array_equal(a.A, c.A)


def test_type1_ranges():
    bt = lpgen.config(2, range(20))
    assert bt.uniform and bt.m[0] == 100 and bt.n[0] == 100
    assert bt.A.min() >= 1.0 and bt.A.max() < 10.0
    assert bt.b.min() >= 10.0 and bt.b.max() < 100.0
    assert bt.c.min() >= 1.0 and bt.c.max() < 10.0
    assert abs(bt.A.mean() - 5.5) < 0.05
    assert (bt.sense == 0).all()


def test_type2_interior_point():
    bt = lpgen.config(3, range(3))
    for k in range(3):
        lp = bt.lp(k)
        assert (lp["sense"][:100] == 0).all() and (lp["sense"][100:] == 1).all()
        # Both row families are built around x0 with margins in [1, 10): the
        # ">=" rows must have b well below the "<=" rows' b on average.
        assert lp["b"][100:].mean() < lp["b"][:100].mean() + 100


def test_config4_mix():
    bt = lpgen.config(4, range(2000))
    frac = np.bincount(bt.gen_type, minlength=4)[1:] / 2000
    assert abs(frac[0] - 0.4) < 0.05 and abs(frac[1] - 0.4) < 0.05 and abs(frac[2] - 0.2) < 0.05
    sim = bt.kind == 0
    assert bt.m[sim].min() >= 5 and bt.m[sim].max() <= 300
    assert bt.n.min() >= 5 and bt.n.max() <= 300
    assert (bt.m[~sim] == 0).all()
    box = np.where(~sim)[0][0]
    lp = bt.lp(int(box))
    assert (lp["l"] < -0.99).all() and (lp["u"] > 0.99).all()


def test_config5_unit_objectives():
    bt = lpgen.config(5, range(50), part="box28")
    c = bt.c.reshape(50, 28)
    assert np.allclose(np.linalg.norm(c, axis=1), 1.0, atol=1e-14)
    s = lpgen.config(5, range(50), part="simplex")
    assert (s.m == s.n).all() and s.m.min() >= 20 and s.m.max() <= 150
    w = lpgen.weights(1005, range(100))
    assert w.min() >= 0.0 and w.max() < 1.0
