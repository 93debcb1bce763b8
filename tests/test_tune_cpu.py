"""The launch-plan tuner's search and cache on the CPU (a synthetic cost
instead of GPU timings)."""
import json

from paper_2112_06396_amd import tune


def _cost(best):
    """Separable cost with its minimum at `best`; one field interacts."""
    def measure(plan):
        t = 100e-6
        for k, v in plan.items():
            if v != best[k]:
                t += 5e-6 * (1 + list(tune.CANDIDATES[k]).index(v) % 3)
        # an interaction: the best conv_group_limbs pays off only with target groups enabled
        if plan["conv_group_max_batch"] == 0 and plan["conv_group_limbs"] == best["conv_group_limbs"]:
            t += 2e-6
        return t
    return measure


def _default():
    return {"e16_fwd_cols": 6144, "e16_fwd_rows": tune.ALWAYS8, "e16_inv_rows": 6144, "e16_inv_cols": 6144,
            "conv_group_limbs": 8, "conv_group_max_batch": 2, "row_xcd_order": 1, "ksk_xcd_order": 1,
            "n1": 0, "col_lines": 16, "row_lines": 8}


def test_descent_finds_the_minimum_of_a_separable_cost():
    best = {"e16_fwd_cols": 0, "e16_fwd_rows": tune.ALWAYS8, "e16_inv_rows": 4096, "e16_inv_cols": 6144,
            "conv_group_limbs": 16, "conv_group_max_batch": 4, "row_xcd_order": 0, "ksk_xcd_order": 1,
            "n1": 0, "col_lines": 32, "row_lines": 4}
    plan, t, t0, trace = tune.coordinate_descent(_cost(best), _default())
    assert plan == best
    assert abs(t - 100e-6) < 1e-12 and t0 > t
    # every measured plan differs from its incumbent in one field
    assert all(set(p) == set(best) for p, _ in trace)


def test_descent_keeps_the_start_when_nothing_is_faster():
    start = _default()
    plan, t, t0, trace = tune.coordinate_descent(_cost(start), start)
    assert plan == start and t == t0
    # one pass over every other candidate value, then stop
    assert len(trace) == 1 + sum(len(v) - 1 for v in tune.CANDIDATES.values())


def test_descent_ignores_gains_below_the_threshold():
    start = _default()

    def measure(plan):  # 0.5% faster with row_xcd_order 0: noise-sized
        return 100e-6 * (0.995 if plan["row_xcd_order"] == 0 else 1.0)
    plan, _, _, _ = tune.coordinate_descent(measure, start, min_gain=0.01)
    assert plan == start


def test_cache_round_trip_and_key(tmp_path):
    path = str(tmp_path / "plans.json")
    assert tune.load_cache(path) == {}
    key = tune.cache_key("gfx950:sramecc+:xnack-", 16, 24, 8, 3, "rotate_l24")
    assert key == "gfx950/n16/L24/K8/d3/rotate_l24"
    e1 = {"plan": _default(), "us": 190.0, "default_us": 192.0, "plans_timed": 30, "outputs_equal": True}
    tune.save_entry(key, e1, path)
    e2 = dict(e1, us=180.0)
    tune.save_entry("gfx950/n16/L24/K8/d3/batch16_l24", e2, path)
    data = tune.load_cache(path)
    assert data[key] == e1 and data["gfx950/n16/L24/K8/d3/batch16_l24"] == e2
    tune.save_entry(key, e2, path)  # replace
    assert tune.load_cache(path)[key]["us"] == 180.0
    json.loads(open(path).read())


def test_candidate_fields_are_the_plan_fields():
    from paper_2112_06396_amd import hks
    assert set(tune.CANDIDATES) == set(hks.PLAN_FIELDS)
    assert all(v in tune.CANDIDATES[k] for k, v in _default().items())


def test_split_candidates_follow_the_ring_degree():
    """The NTT split candidates keep both passes within 5..9 stages."""
    assert tune.candidates_for(16)["n1"] == (0, 7, 9)
    assert tune.candidates_for(15)["n1"] == (0, 6, 8)
    assert tune.candidates_for(10)["n1"] == (0,)
    assert tune.candidates_for(12)["n1"] == (0, 5, 7)


def test_committed_plans_are_valid():
    """Every plan in the package's cache names only plan fields with values
    the library accepts."""
    from paper_2112_06396_amd import hks
    for key, entry in tune.load_cache().items():
        plan = entry["plan"]
        assert set(plan) == set(hks.PLAN_FIELDS), key
        assert 1 <= plan["conv_group_limbs"] <= 64
        assert plan["row_xcd_order"] in (0, 1) and plan["ksk_xcd_order"] in (0, 1)
        assert plan["col_lines"] in (8, 16, 32) and plan["row_lines"] in (4, 8, 16)
        assert entry["outputs_equal"] and entry["us"] <= entry["default_us"]
