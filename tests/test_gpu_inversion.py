"""Surrogate-assisted c^2 inversion against BBWADG-only inversion, through the C ABI.

Workload: the 16^3 x 6 Kuhn cube (24,576 tets), N = 4, M = 2, rigid walls, a Gaussian pulse
at (0.5, 0.5, 0.85), 64 receivers on the top face, 200 LSRK4 steps. The surrogate is trained
on the traces of 128 seeded random media (2,000 Adam steps); the true medium is another
seeded medium of the same family, written as a linear combination of its layer indicators
and bumps, and the inversion starts from the mean layer value with no bumps.

Both runs start from the same parameters and stop at the same misfit reduction. The gain is
the wall time to that reduction, the surrogate's training excluded (it is paid once for any
number of inversions in the family). Every misfit on the path is BBWADG's own (the check), and
every accepted surrogate round has a relative trace error at most `max_err` there."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CELLS, N, M, NSTEPS = 16, 4, 2, 200
NMOD, TRAIN_STEPS, MAX_ERR, TARGET = 128, 2000, 0.2, 0.3


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1808_08645_amd as bb
    from paper_1808_08645_amd.surrogate import Surrogate
    from workloads import c2_random_model, grid_centres, ic_gaussian_pulse, kuhn_cube_mesh, receiver_grid
    print("[inversion] training data and surrogate", flush=True)
    xyz, etov = kuhn_cube_mesh(CELLS)
    s = bb.Solver(xyz, etov, N, M, dtype="f64", bc="rigid")
    s.set_receivers(receiver_grid(8, 1.0))
    pulse = lambda x, y, z: ic_gaussian_pulse(x, y, z, centre=(0.5, 0.5, 0.85), width=0.1)  # noqa: E731
    zero = lambda x, y, z: 0.0 * x  # noqa: E731
    q0 = s.to_device(s.initial_state([pulse, zero, zero, zero]))
    s.project_c2(lambda x, y, z: 4.0 + 0.0 * x)
    dt = s.suggest_dt(0.5)  # CFL 0.5 at the largest c^2 of the family
    gx, gy, gz = grid_centres(16)
    X = np.zeros((NMOD, 16, 16, 16), np.float32)
    Y = np.zeros((NMOD, NSTEPS * 64), np.float32)
    for i in range(NMOD):
        f = c2_random_model(i)
        X[i] = f(gx, gy, gz)
        s.project_c2(f)
        _, _, tr = s.misfit_gradient(q0, dt, NSTEPS, None, gradient=False)
        Y[i] = tr.cpu().numpy().ravel()
    sigma = float(Y.std())
    sur = Surrogate(NSTEPS * 64, 32, seed=1)
    xd = torch.tensor((X - 2.5) / 1.5, device="cuda")
    yd = torch.tensor(Y / sigma, device="cuda")
    rng = np.random.default_rng(2)
    for k in range(TRAIN_STEPS):
        idx = torch.tensor(rng.choice(NMOD, 32, replace=False), device="cuda")
        sur.train_step(xd[idx], yd[idx], 1e-5 + 0.5 * (1e-3 - 1e-5) * (1 + np.cos(np.pi * k / TRAIN_STEPS)))
    torch.cuda.synchronize()
    return s, q0, dt, sur, sigma


def _time_to(hist, level):
    hit = [h["t"] for h in hist if h["J"] <= level]
    return hit[0] if hit else None


SEEDS = (1000, 1001, 1002)


def test_surrogate_inversion_reaches_misfit_reduction_sooner(setup):
    """Per true medium: both runs reach J <= TARGET J0 from the same start; every accepted
    surrogate round had trace error <= MAX_ERR; where the surrogate's first round was kept,
    it got there sooner; where the rule fell back at once, the rest of its run is the
    BBWADG-only run (same misfits), late by the rejected rounds only. Over the family the
    surrogate-assisted runs take less time in total."""
    from paper_1808_08645_amd.inversion import Inversion, LinearMedium
    from workloads import c2_random_model_family, grid_centres
    s, q0, dt, sur, sigma = setup
    tot_sur = tot_bb = 0.0
    for seed in SEEDS:
        print(f"[inversion] true medium seed {seed}", flush=True)
        phis, th_true = c2_random_model_family(seed)
        med = LinearMedium(s, phis, grid_centres(16))
        s.set_c2(med.coef(th_true))
        _, _, d = s.misfit_gradient(q0, dt, NSTEPS, None, gradient=False)
        data = d.cpu().numpy()
        nl = len(th_true) - 4
        th0 = th_true.copy()
        th0[:nl] = th_true[:nl].mean()
        th0[nl:] = 0.0
        hists = {}
        for name, use in (("surrogate", True), ("bbwadg", False)):
            inv = Inversion(s, med, q0, dt, NSTEPS, data, surrogate=sur if use else None, sigma=sigma)
            _, hists[name] = inv.run(th0, max_time=60.0, target=TARGET, max_err=MAX_ERR)
        hs, hb = hists["surrogate"], hists["bbwadg"]
        J0 = hb[0]["J"]
        assert hs[0]["J"] == pytest.approx(J0, rel=1e-12)  # same start, same check
        t_sur, t_bb = _time_to(hs, TARGET * J0), _time_to(hb, TARGET * J0)
        rounds = [h for h in hs if h["kind"] == "surrogate round"]
        print(f"[inversion] seed {seed}: time to J <= {TARGET} J0: surrogate {t_sur:.3f} s "
              f"({sum(h['accepted'] for h in rounds)} of {len(rounds)} surrogate rounds kept), "
              f"BBWADG {t_bb:.3f} s", flush=True)
        assert t_sur is not None and t_bb is not None
        assert all(h["surrogate_err"] <= MAX_ERR for h in rounds if h["accepted"])
        if rounds[0]["accepted"]:
            assert t_sur < t_bb
        else:
            # fell back before moving: from then on the BBWADG-only path, misfit for misfit
            after = [h["J"] for h in hs if h["kind"] != "surrogate round"]
            assert after == pytest.approx([h["J"] for h in hb][:len(after)], rel=1e-12)
        for hist in (hs, hb):  # kept misfits are BBWADG's and never increase
            Js = [h["J"] for h in hist]
            assert all(b <= a for a, b in zip(Js, Js[1:]))
        tot_sur += t_sur
        tot_bb += t_bb
    print(f"[inversion] total time to J <= {TARGET} J0 over {len(SEEDS)} media: surrogate {tot_sur:.3f} s, "
          f"BBWADG {tot_bb:.3f} s", flush=True)
    assert tot_sur < tot_bb
