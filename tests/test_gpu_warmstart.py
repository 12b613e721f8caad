"""Learned warm start on the GPU: trained on the solver's own solutions, judged by the solver.
The trained network must cut the iterations of held-out instances against the cold start while
reaching the same KKT points; unusable warm points fall back to the cold start."""
import numpy as np
import pytest

import oracle
from paper_2606_26341_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def trained(torch_cuda):
    from paper_2606_26341_amd import warmstart
    w = W.get("C5")
    ws, losses, n = warmstart.train_for(w, 16384, seed_tag=51, epochs=30, batch=1024)
    say("trained on", n, "solutions; loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.2 * losses[0]
    return w, ws


def test_warm_start_cuts_iterations(torch_cuda, trained):
    torch = torch_cuda
    from paper_2606_26341_amd import hipipm
    w, ws = trained
    TH = torch.tensor(w.thetas(0, 2048), dtype=torch.float64, device="cuda")
    # the warm barrier parameter the validation split picks for this network (1e-4)
    s = hipipm.Solver(w, 2048, hipipm.default_options(warm_mu0=1e-4))
    cold = {k: v.cpu().numpy() for k, v in s.solve(TH).items()}
    warm_pts = ws.predict(TH)
    s.reset_stats()
    warm = {k: v.cpu().numpy() for k, v in s.solve(TH, warm=warm_pts).items()}
    st = s.stats()
    okc, okw = cold["status"] == 1, warm["status"] == 1
    say("cold: converged", okc.mean(), "mean iters", cold["iters"].mean(),
        "| warm: converged", okw.mean(), "mean iters", warm["iters"].mean(), "stats", st)
    # the gate sends some rows of this small-sample network back to the cold start (about 11 %;
    # none of the 190,000-solution network's rows on the same distribution)
    assert st["warm_started"] == 2048 and st["warm_rejected"] <= 0.25 * 2048
    assert okw.mean() >= okc.mean() - 0.01
    assert warm["iters"][okw].mean() < 0.8 * cold["iters"][okc].mean()
    both = okc & okw
    rel = np.abs(warm["obj"] - cold["obj"]) / np.maximum(1.0, np.abs(cold["obj"]))
    same = both & (rel <= 1e-6) & (np.abs(warm["x"] - cold["x"]).max(axis=1) <= 1e-5)
    say("same KKT point", same.sum(), "of", both.sum())
    assert same.sum() >= 0.9 * both.sum()
    for i in np.flatnonzero(okw)[:8]:
        th = TH[i].cpu().numpy()
        assert oracle.kkt_error(w, th, warm["x"][i], warm["y"][i], warm["zl"][i], warm["zu"][i]) <= 1e-8


def test_unusable_warm_points_fall_back_to_cold(torch_cuda, trained):
    torch = torch_cuda
    from paper_2606_26341_amd import hipipm
    w, ws = trained
    TH = torch.tensor(w.thetas(5000, 64), dtype=torch.float64, device="cuda")
    for gate in (0, 1):
        s = hipipm.Solver(w, 64, hipipm.default_options(warm_iter_cap=40, warm_gate=gate))
        cold = {k: v.cpu().numpy() for k, v in s.solve(TH).items()}
        bad = ws.predict(TH)
        bad[0:16, 5] = float("nan")                     # rejected at initialisation
        bad[16:32] = bad[16:32] * 0.0 + 50.0            # far from anything: rejected by the gate, or
        s.reset_stats()                                 # restarted cold, or still converging
        out = {k: v.cpu().numpy() for k, v in s.solve(TH, warm=bad).items()}
        st = s.stats()
        say("gate", gate, "stats", st, "statuses", np.bincount(out["status"]))
        if gate:
            # the 32 unusable rows, and any network row whose E_mu0 is above the cold start's
            assert st["warm_rejected"] >= 32
            for k in ("x", "y", "zl", "zu", "obj", "kkt", "status", "iters"):
                assert np.array_equal(out[k][:32], cold[k][:32]), k    # those 32 solve exactly as cold
        else:
            assert st["warm_rejected"] == 16
        assert (out["status"][0:16] == cold["status"][0:16]).all()
        assert (out["status"] == 1).mean() >= (cold["status"] == 1).mean() - 0.05


def _warm_rows(ws, TH):
    rows = ws.predict(TH).cpu().numpy()
    rows[16:24] += 40.0                  # far worse than the cold start: the gate rejects them
    rows[24:28, 3] = float("nan")        # non-finite: rejected before the gate
    return rows


def test_warm_initial_state_matches_oracle(torch_cuda, trained):
    """The warm initialisation on both sides: after the INIT_Y passes (with the gate, the cold start's
    least-squares pass, then the warm point's pass with multipliers from stationarity and the E_mu0
    comparison) the GPU slot states equal the oracle's, element by element (e_v <= 1e-8, the same
    phase, iteration count and warm flag); one pass later (the first iteration) as well."""
    torch = torch_cuda
    from paper_2606_26341_amd import hipipm
    from helpers import compare_states
    w, ws = trained
    th = w.thetas(7000, 48)
    TH = torch.tensor(th, dtype=torch.float64, device="cuda")
    rows = _warm_rows(ws, TH)
    WR = torch.tensor(rows, dtype=torch.float64, device="cuda")
    s = hipipm.Solver(w, th.shape[0], hipipm.default_options())
    s.start(TH, WR)
    hs = [oracle.Handle.quad(w, th[i], warm_row=rows[i]) for i in range(th.shape[0])]
    for passes in (2, 1):
        s.step(th.shape[0], passes, TH, WR)
        g = s.state_export(th.shape[0])
        worst = 0.0
        n_warm = 0
        for i, h in enumerate(hs):
            for _ in range(passes):
                h.step()
            so = h.state()
            bad, ev = compare_states(g[i], so, w.n, w.m)
            fo = oracle.unpack_state(so, w.n, w.m)
            fg = oracle.unpack_state(g[i], w.n, w.m)
            assert not bad, (i, bad)
            assert fg["warm"] == fo["warm"], (i, fg["warm"], fo["warm"])
            n_warm += fo["warm"]
            worst = max(worst, ev)
        say("after", passes, "more passes: warm", n_warm, "of", len(hs), "worst e_v", worst)
        assert worst <= 1e-8
        assert 0 < n_warm <= len(hs) - 12


@pytest.mark.parametrize("precision", [0, 1])
def test_warm_solves_match_oracle(torch_cuda, trained, precision):
    """Network-warm-started solves (gate on; FP64, and FP32 + FP64 refinement as in the warm/mixed
    benchmark) against the oracle's warm solves from the same rows: same status, the same KKT point
    (relative objective <= 1e-6, |x - x*|_inf <= 1e-5) and E_0 <= 1e-8 re-checked by the oracle."""
    torch = torch_cuda
    from paper_2606_26341_amd import hipipm
    w, ws = trained
    th = w.thetas(8000, 64)
    TH = torch.tensor(th, dtype=torch.float64, device="cuda")
    rows = _warm_rows(ws, TH)
    s = hipipm.Solver(w, 24, hipipm.default_options(precision=precision))
    g = {k: v.cpu().numpy() for k, v in s.solve(TH, warm=torch.tensor(rows, dtype=torch.float64,
                                                                             device="cuda")).items()}
    st = s.stats()
    o = oracle.solve_quad(w, th, threads=16, warm=rows)
    say("gpu stats", st, "oracle warm started / rejected", o["stats"][:, 8].sum(), o["stats"][:, 9].sum())
    assert st["warm_started"] == int(o["stats"][:, 8].sum())
    assert st["warm_rejected"] == int(o["stats"][:, 9].sum())
    assert (g["status"] == o["status"]).all()
    if precision == 0:
        assert np.array_equal(g["iters"], o["iters"])
    for i in np.flatnonzero(o["status"] == oracle.ST_CONVERGED):
        rel = abs(g["obj"][i] - o["obj"][i]) / max(1.0, abs(o["obj"][i]))
        assert rel <= 1e-6 and np.abs(g["x"][i] - o["x"][i]).max() <= 1e-5, i
        assert oracle.kkt_error(w, th[i], g["x"][i], g["y"][i], g["zl"][i], g["zu"][i]) <= 1e-8, i


def test_warm_start_at_the_oracle_solution_converges_at_once(torch_cuda):
    """Special case: started from the oracle's own converged (w, y) with a barrier parameter of 1e-6
    the method is already at the solution up to the barrier term; it must finish within three
    iterations at the oracle's KKT point."""
    torch = torch_cuda
    from paper_2606_26341_amd import hipipm
    w = W.get("C1")
    th = w.thetas(0, w.n_inst)
    o = oracle.solve_quad(w, th, threads=8)
    assert (o["status"] == oracle.ST_CONVERGED).all()
    TH = torch.tensor(th, dtype=torch.float64, device="cuda")
    warm = torch.tensor(np.concatenate([o["x"][:, :w.n_w], o["y"]], axis=1), dtype=torch.float64, device="cuda")
    s = hipipm.Solver(w, w.n_inst, hipipm.default_options(warm_mu0=1e-6))
    out = {k: v.cpu().numpy() for k, v in s.solve(TH, warm=warm).items()}
    say("iterations", np.bincount(out["iters"]), "stats", s.stats())
    assert (out["status"] == 1).all() and out["iters"].max() <= 3
    rel = np.abs(out["obj"] - o["obj"]) / np.maximum(1.0, np.abs(o["obj"]))
    assert rel.max() <= 1e-6 and np.abs(out["x"] - o["x"]).max() <= 1e-5 and out["kkt"].max() <= 1e-8
