"""GPU test of the tile autotuner through the C ABI: a tuning run records a tile per product-launch
shape; plans built from the tuned table reproduce the oracle's operator; the table round-trips
through its JSON cache.  The table is process-wide, so the test empties it when done."""
import numpy as np
import pytest

from oracle import nd_dtn
from parity import assert_close

pytestmark = pytest.mark.gpu


@pytest.fixture
def fresh_table(dtn):
    dtn.tune_clear()
    dtn.tune_enable(True)
    yield
    dtn.tune_clear()
    dtn.tune_enable(True)


def test_tuned_plans_reproduce_the_oracle(dtn, fresh_table, tmp_path):
    n, leaf = 300, 32
    rng = np.random.default_rng(17)
    b, c, d = rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    rep = dtn.tune(n, b, c, d, leaf=leaf, reps=1)
    assert len(rep) > 0 and dtn.tune_size() == len(rep)
    assert all(v["tile"] in (0, 2, 3, 4) for v in rep.values())
    # the chosen tile is the fastest, or the thresholds' own tile when within 3 % of it
    for sig, v in rep.items():
        best = min(v["ms"], key=lambda t: v["ms"][t])
        assert int(best) == v["tile"] or (v["tile"] == v["default"] and
                                           v["ms"][str(v["default"])] <= 1.03 * v["ms"][best]), (sig, v)
    Tref = nd_dtn(n, b, c, d, leaf=leaf)
    tuned = dtn.build(n, b, c, d, leaf=leaf).dense()
    assert_close(tuned, Tref, 1e-10, label="tuned plan vs oracle")
    dtn.tune_enable(False)
    default = dtn.build(n, b, c, d, leaf=leaf).dense()
    assert_close(default, Tref, 1e-10, label="fixed-threshold plan vs oracle")
    assert_close(tuned, default, 1e-13, label="tuned vs fixed-threshold plan")
    dtn.tune_enable(True)
    path = tmp_path / "tune.json"
    dtn.tune_save(str(path))
    dtn.tune_clear()
    dtn.tune_load(str(path))
    assert dtn.tune_size() == len(rep)
    again = dtn.build(n, b, c, d, leaf=leaf).dense()
    assert np.array_equal(again, tuned)
