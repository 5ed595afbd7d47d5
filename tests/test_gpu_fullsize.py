"""Full-size workloads on the GPU, checked by the FP64 oracle on the returned
state (needs an MI355X).

At these sizes the oracle cannot run the iteration itself, so each check
re-measures what holds at any size: the stopping sum of the GPU's returned
potentials over every node (computed by the oracle in FP64 from those
potentials), the GPU's own FP64 evaluation against the oracle's evaluation
of the same potentials, unit mass of every plan (Lemma tree_mass) and the
duality-gap bound |P - D| <= C_inf E."""
import numpy as np
import pytest

from oracle import TreeOracle
from workloads import make_config, make_batched_stars

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


def check_state(g, p, tol):
    o = TreeOracle(p)
    lam = o.set_potentials(g.potentials())
    e_sum, _ = o.full_error(lam)
    assert e_sum <= tol + 1e-10, e_sum
    eg = g.evaluate()
    assert abs(eg["err_sum"] - e_sum) <= 1e-9
    assert abs(eg["mass_min"] - 1.0) <= 1e-9 and abs(eg["mass_max"] - 1.0) <= 1e-9
    assert abs(eg["gap"]) <= o.c_inf() * eg["err_sum"] + 1e-12
    return e_sum, eg


def test_random_tree_256_nodes_2d_converges(ctx):
    """256-node Pruefer tree, n in [256, 4096] on 2D grids, eps = 5e-3, solved
    to 1e-6 (separable grid passes), re-measured by the oracle and compared
    with the oracle's state at a stopping sum of 1e-9
    (tests/golden/random_tree256_converged.json, written by
    make_tree_golden.py, which calls only the oracle): both duals lie within
    2 C_inf E of the optimum (Lemma f_upper_bound_tree), so they agree to 1e-6
    of the scale and to 2 C_inf (E_gpu + E_ref); primals to 3 C_inf (...)."""
    import json
    import os
    from paper_2406_10849_amd import Problem
    p = make_config(3)
    g = Problem(ctx, p)
    r = g.solve(tol=1e-6, max_steps=200000)
    assert r["status"] == "converged"
    _, ev = check_state(g, p, 1e-6)
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "random_tree256_converged.json")))
    assert ref["err_sum"] <= 1e-9
    assert abs(ev["dual"] - ref["dual"]) <= 1e-6 * ref["scale"]
    assert abs(ev["dual"] - ref["dual"]) <= 2 * ref["c_inf"] * (ev["err_sum"] + ref["err_sum"])
    assert abs(ev["primal"] - ref["primal"]) <= 3 * ref["c_inf"] * (ev["err_sum"] + ref["err_sum"])


def test_batched_512_stars_sampled(ctx):
    """512 uneven stars in one batch, the benchmark's launch configuration;
    8 sampled instances re-measured by the oracle, and the 12 instances of
    tests/golden/batched_stars_sample_converged.json (oracle only, stopping
    sum <= 1e-10, make_batched_golden.py) compared with their converged dual:
    both duals lie within 2 C_inf E of the optimum (Lemma f_upper_bound_tree),
    so they agree to 1e-6 of the scale and to 2 C_inf (E_gpu + E_ref)."""
    import json
    import os
    from paper_2406_10849_amd import Batch, Problem
    probs = make_batched_stars(count=512)
    gps = [Problem(ctx, p) for p in probs]
    b = Batch(ctx, gps)
    b.autotune()
    rs = b.solve(tol=1e-6, max_steps=200000, check_every=16)
    assert all(r["status"] == "converged" for r in rs)
    rng = np.random.default_rng(0)
    for i in rng.choice(len(probs), size=8, replace=False):
        check_state(gps[i], probs[i], 1e-6)
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batched_stars_sample_converged.json")))
    assert len(ref["instances"]) == 12
    for rec in ref["instances"]:
        i = rec["index"]
        assert probs[i].name == rec["name"]
        ev = gps[i].evaluate()
        assert ev["err_sum"] <= 1e-6
        assert abs(ev["dual"] - rec["dual"]) <= 1e-6 * rec["scale"], (i, ev["dual"], rec["dual"])
        assert abs(ev["dual"] - rec["dual"]) <= 2 * rec["c_inf"] * (ev["err_sum"] + rec["err_sum"]), i
        assert abs(ev["primal"] - rec["primal"]) <= 3 * rec["c_inf"] * (ev["err_sum"] + rec["err_sum"]), i


def test_chain_dual_matches_converged_reference():
    """32-node chain (n = 1024, eps = 1e-3), solved to a stopping sum of 1e-6
    on the device, against the FP64 oracle's state at a stopping sum of 1e-10
    (tests/golden/chain32_n1024_converged.json, written by make_chain_golden.py,
    which calls only the oracle).  Both duals are within 2 C_inf E of the
    optimum (Lemma f_upper_bound_tree), so they agree to 1e-6 of the scale;
    primals are within C_inf E of their duals, so they agree to
    3 C_inf (E_gpu + E_ref)."""
    import json
    import os
    from paper_2406_10849_amd import Context, Problem
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "chain32_n1024_converged.json")))
    p = make_config(2)
    g = Problem(Context(0), p)
    r = g.solve(tol=1e-6, max_steps=200000)
    assert r["status"] == "converged"
    ev = g.evaluate()
    assert ev["err_sum"] <= 1e-6
    assert abs(ev["dual"] - ref["dual"]) <= 1e-6 * ref["scale"]
    assert abs(ev["dual"] - ref["dual"]) <= 2 * ref["c_inf"] * (ev["err_sum"] + ref["err_sum"])
    assert abs(ev["primal"] - ref["primal"]) <= 3 * ref["c_inf"] * (ev["err_sum"] + ref["err_sum"])
