"""CPU checks of the autotuner's host logic and the learned predictor."""
import json
import math

import numpy as np

from paper_2003_03868_amd import tune


def test_committed_table_is_complete_and_valid():
    tab = tune.load_table()
    assert len(tab) == 29 ** 3 + 16
    for (m, n, k), e in tab.items():
        assert e in tune.entries_for(m, n, k), ((m, n, k), e)
    # the compile-time-shape kernel won every uniform shape it exists for
    for b in tune.FIXED_SIZES:
        assert tab[(b, b, b)] == tune.FIXED_ENTRY


def test_model_choices_are_valid_entries():
    model = json.load(open(tune.MODEL_PATH))
    keys = [(4, 4, 4), (23, 23, 23), (5, 26, 0), (31, 7, 19)]
    tab = tune.table_from_model(model, keys)
    for key in keys:
        assert tab[key] in tune.entries_for(*key)
        assert tab[key] == tune.predict(model, *key, 60000, 32)
    # with the exhaustive table as fallback, undecided keys take its entry
    exh = tune.load_table()
    tab2 = tune.table_from_model(model, keys, fallback=exh)
    for key in keys:
        want = tab[key] if key in tune.table_from_model.trusted else exh[key]
        assert tab2[key] == want


def test_ensemble_trust_and_fallback():
    """An ensemble whose members disagree on a shape falls back to the
    exhaustive best there (regret 0), and agrees with its members where they
    agree."""
    rng = np.random.default_rng(4)
    recs = _synthetic_records(rng, 200)
    model, rep = tune.train_ensemble(recs, members=3, epochs=60)
    assert len(tune.members_of(model)) == 3
    te = tune.split_triples(recs)[1]
    assert rep["test_with_fallback"]["mean"] <= rep["test_ensemble"]["mean"] + 1e-12
    assert 0.0 <= rep["trusted_share_test"] <= 1.0
    r = te[0]
    picks = {tune.predict(m, r["m"], r["n"], r["k"], r["n_c"] * r["per_c"], r["per_c"])
             for m in tune.members_of(model)}
    if len(picks) == 1:
        assert tune.predict(model, r["m"], r["n"], r["k"], r["n_c"] * r["per_c"], r["per_c"]) in picks


def test_operand_reuse_feature():
    """The occupancy input: products per operand block of the stack."""
    assert tune.operand_reuse(2048 * 8, 13) == 8.0
    assert tune.operand_reuse(2048 * 8 * 4, 0) == 8.0
    f = tune.features(23, 23, 23, 60000, 32)
    assert len(f) == 9 and abs(f[-1] - math.log2(60000 / 2048) / 8.0) < 1e-12


def _synthetic_records(rng, n_triples=300):
    """Timings where the best entry is a known function of the shape."""
    recs = []
    for _ in range(n_triples):
        m, n, k = (int(v) for v in rng.integers(4, 33, 3))
        ents = tune.entries_for(m, n, k)
        ms = []
        for f, w, p in ents:
            t = 1.0 + 0.3 * f * (m % 16 == 0) + 0.5 * (1 - f) * (m % 16 != 0) + 0.1 * (w != 1) - 0.05 * p
            ms.append(t * (1 + 0.01 * rng.random()))
        recs.append(dict(m=m, n=n, k=k, n_c=1875, per_c=32, entries=[list(e) for e in ents], ms=ms))
    return recs


def test_training_learns_a_known_rule():
    # 600 triples: the rule turns on m = 16, 32, so a smaller held-out set
    # may hold almost none of them
    rng = np.random.default_rng(0)
    recs = _synthetic_records(rng, 600)
    model, rep = tune.train(recs, epochs=150, seed=1)
    assert rep["test"]["mean"] < 0.05
    assert rep["test"]["mean"] < tune.default_regret(tune.split_triples(recs)[1], (0, 2, 0))["mean"]


def test_regret_and_split():
    recs = _synthetic_records(np.random.default_rng(2), 50)
    tr, te, held = tune.split_triples(recs, 0.2, 0)
    assert not ({(r["m"], r["n"], r["k"]) for r in tr} & held)
    best = [min(r["ms"]) for r in recs]
    assert all(b > 0 for b in best)
    d = tune.default_regret(recs, (1, 1, 1))
    assert d["mean"] >= 0 and math.isfinite(d["max"])
