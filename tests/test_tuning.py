"""Host logic of the tuning table (paper_1504_05090_amd.tuning): the
committed gfx950 table covers the multigrid workload, lookups match on
every key, and apply() sets per-instance parameters only where an entry
exists."""
from paper_1504_05090_amd import tuning
from paper_1504_05090_amd.workloads import BASE_SEED, CONFIGS, T_HOP


def c3_instances():
    w = CONFIGS["C3"]
    return [dict(L=q["L"], U=q["U"], t=T_HOP, beta=q["beta"], dtau=q["dtau"], seed=BASE_SEED, n_chains=w["chains"])
            for q in w["instances"]]


def test_table_covers_the_multigrid_workload():
    entries = tuning.load("gfx950")
    assert entries, "no committed gfx950 table"
    for d in c3_instances():
        hit = tuning.lookup(d, "fp64", arch="gfx950", entries=entries)
        assert hit is not None, d
        k, ns = hit
        assert 1 <= k <= 32 and 1 <= ns <= round(d["beta"] / d["dtau"])
    for e in entries:
        assert e["met_bound"] == 1 and e["drift_rel_max"] <= e["drift_bound"]


def test_lookup_matches_every_key():
    d = c3_instances()[-1]
    entries = tuning.load("gfx950")
    assert tuning.lookup(d, "fp64", arch="gfx950", entries=entries) is not None
    for change in (dict(L=14), dict(U=3.0), dict(t=0.3), dict(dtau=0.25, beta=20.0)):
        assert tuning.lookup(dict(d, **change), "fp64", arch="gfx950", entries=entries) is None, change
    assert tuning.lookup(d, "mixed", arch="gfx950", entries=entries) is None
    assert tuning.lookup(d, "fp64", arch="gfx942", entries=[]) is None


def test_apply_sets_parameters_only_where_tuned():
    insts = c3_instances()[:2] + [dict(L=4, U=2.0, t=T_HOP, beta=4.0, dtau=0.5, seed=1, n_chains=1)]
    out = tuning.apply(insts, "fp64", arch="gfx950")
    assert [d["tuned"] for d in out] == [True, True, False]
    assert "delay_k" not in out[2] and "n_stab" not in out[2]
    for d in out[:2]:
        assert (d["delay_k"], d["n_stab"]) == tuning.lookup(d, "fp64", arch="gfx950")
    assert "tuned" not in insts[0]   # the inputs are left alone
