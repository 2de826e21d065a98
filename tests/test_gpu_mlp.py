"""GPU parity of the learned warm start: forward and backward MFMA kernels and Adam
against the oracle (bf16 emulated at the same points), and the ROW3 warm start
trained on stage solves the method logs."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
from oracle import mlp as omlp
from tests.gpu_common import rel, setup, to_gpu, to_np, vortex_state

pytestmark = pytest.mark.gpu


def _params_from_master(tr):
    m = tr.master.detach().cpu().numpy().astype(np.float64)
    In, H, Out = tr.net.n_in, tr.net.n_hidden, tr.net.n_out
    p, o = {}, 0
    for name, (r, c) in (("1", (H, In)), ("2", (H, H)), ("3", (Out, H))):
        p["W" + name] = m[o:o + r * c].reshape(r, c)
        o += r * c
        p["b" + name] = m[o:o + r]
        o += r
    return p


def _trainer(P=3, H=256, seed=4):
    from paper_1904_04825_amd import MlpTrainer
    _, op, disc = setup(6, 5, P, "rusanov")
    tr = MlpTrainer(disc, n_hidden=H, seed=seed)
    m = tr.master.cpu().numpy()
    rng = np.random.default_rng(9)
    p = _params_from_master(tr)   # put non-zero biases in
    o = 0
    for name in ("1", "2", "3"):
        o += p["W" + name].size
        m[o:o + p["b" + name].size] = 0.05 * rng.standard_normal(p["b" + name].size)
        o += p["b" + name].size
    tr.set_master(m)
    return disc, tr


@pytest.mark.parametrize("P", [2, 3])
def test_mlp_forward_parity(P):
    disc, tr = _trainer(P)
    X = np.random.default_rng(1).standard_normal((300, tr.net.n_in))
    Xb = torch.as_tensor(X, dtype=torch.float32, device="cuda").to(torch.bfloat16)
    y = tr.net.forward(Xb).cpu().numpy()
    yo, _ = omlp.forward(_params_from_master(tr), X, emulate_bf16=True)
    print(f"P={P} forward rel {rel(y, yo):.2e}", flush=True)
    assert rel(y, yo) <= 1e-3


def _synthetic_log(disc, count, seed):
    from paper_1904_04825_amd import StageLog
    lg = StageLog(disc, count, np.arange(min(8, disc.nel)))
    rng = np.random.default_rng(seed)
    Np = disc.np_
    mu = rng.uniform(-2, 2, 20)
    sd = rng.uniform(0.1, 3, 20)
    raw = np.concatenate([mu[g] + sd[g] * rng.standard_normal((count, Np)) for g in range(20)], axis=1)
    lg.samples.copy_(torch.as_tensor(raw, dtype=torch.float32))
    lg.c.count = count
    return lg, raw


def test_mlp_stats_gradients_and_adam():
    disc, tr = _trainer(3)
    lg, raw = _synthetic_log(disc, 512, seed=3)
    tr.fit_stats(lg)
    norm = tr.net.norm.cpu().numpy().astype(np.float64)
    Np = disc.np_
    raw32 = raw.astype(np.float32).astype(np.float64)
    ref = np.array([[raw32[:, g * Np:(g + 1) * Np].mean(), raw32[:, g * Np:(g + 1) * Np].std()] for g in range(20)])
    assert np.allclose(norm.reshape(20, 2), ref, rtol=1e-5, atol=1e-6)
    idx = np.random.default_rng(5).choice(512, size=256, replace=False)
    p0 = _params_from_master(tr)
    loss = tr.step(lg, torch.as_tensor(idx, dtype=torch.int32, device="cuda"), lr=0.0)
    # oracle on the same batch: inputs standardised with the device statistics, rounded to bf16
    In = 16 * Np
    mean = norm[0::2].astype(np.float32)
    std = norm[1::2].astype(np.float32)
    Xr = raw32[idx, :In].astype(np.float32)
    X = ((Xr - np.repeat(mean[:16], Np)) / np.repeat(std[:16], Np)).astype(np.float64)
    T = ((raw32[idx, In:].astype(np.float32) - np.repeat(mean[16:], Np)) / np.repeat(std[16:], Np)).astype(np.float64)
    y, cache = omlp.forward(p0, X, emulate_bf16=True)
    assert abs(loss - omlp.mse(y, T)) <= 1e-3 * omlp.mse(y, T)
    g_or = omlp.backward(p0, cache, y, T, emulate_bf16=True)
    g_gpu = {}
    gflat = tr.grad.cpu().numpy().astype(np.float64)
    o = 0
    for name in ("1", "2", "3"):
        w = p0["W" + name]
        g_gpu["W" + name] = gflat[o:o + w.size].reshape(w.shape)
        o += w.size
        g_gpu["b" + name] = gflat[o:o + w.shape[0]]
        o += w.shape[0]
    for k in g_or:
        print(k, f"{rel(g_gpu[k], g_or[k]):.2e}", flush=True)
        assert rel(g_gpu[k], g_or[k]) <= 1e-2 if k.startswith("b") else rel(g_gpu[k], g_or[k]) <= 1e-3
    # one Adam step from the device gradients
    tr.step(lg, torch.as_tensor(idx, dtype=torch.int32, device="cuda"), lr=1e-3)
    p1 = _params_from_master(tr)
    g_used = {}
    gflat = tr.grad.cpu().numpy().astype(np.float64)
    o = 0
    for name in ("1", "2", "3"):
        w = p0["W" + name]
        g_used["W" + name] = gflat[o:o + w.size].reshape(w.shape)
        o += w.size
        g_used["b" + name] = gflat[o:o + w.shape[0]]
        o += w.shape[0]
    p_or = omlp.adam_step({k: v.copy() for k, v in p0.items()}, g_used, {}, lr=1e-3)
    for k in p_or:
        assert np.allclose(p1[k], p_or[k], rtol=1e-5, atol=1e-6), k


def test_row3_learned_warm_start():
    """Log stage solves of the vortex, train one network per ROW3 stage on the GPU,
    then compare GMRES iterations with and without the learned guess."""
    from paper_1904_04825_amd import GmresOpts, MlpTrainer, SolverOpts, StageLog, StageLogs, WarmStart
    _, op, disc = setup(16, 16, 3, "rusanov", seed=2)
    U0 = to_gpu(vortex_state(op, 0.0))
    dt, S = 0.1, 4
    rng = np.random.default_rng(40)
    logs = StageLogs([StageLog(disc, 6000, rng.choice(disc.nel, 200, replace=False)) for _ in range(S)])
    yhist = torch.zeros((2, disc.ndof), dtype=torch.float64, device="cuda")
    U = U0.clone()
    opts = SolverOpts(lin=GmresOpts(m=20, rtol=1e-8), log=logs, yhist=yhist)
    for n in range(24):
        for lg in logs.logs:
            lg.set_elems(rng.choice(disc.nel, 200, replace=False))
        st = disc.row_step(U, 3, dt, opts)
        assert st["status"] == 0
    assert all(lg.count == 24 * 200 for lg in logs.logs)
    trainers = []
    for i, lg in enumerate(logs.logs):
        tr = MlpTrainer(disc, n_hidden=256, seed=4 + i, lr=1e-3)
        tr.fit_stats(lg)
        losses = []
        for it in range(400):
            idx = torch.as_tensor(rng.choice(lg.count, 512, replace=False), dtype=torch.int32, device="cuda")
            losses.append(tr.step(lg, idx))
        print(f"stage {i}: loss {losses[0]:.3e} -> {np.mean(losses[-20:]):.3e}", flush=True)
        assert np.mean(losses[-20:]) < 0.5 * losses[0]
        trainers.append(tr)
    warm = WarmStart([t.net for t in trainers])
    # continue from the logged run: plain and warm steps from the same state
    Up, Uw = U.clone(), U.clone()
    hp, hw = yhist.clone(), yhist.clone()
    it_p = it_w = 0
    used = rej = 0
    for n in range(6):
        sp = disc.row_step(Up, 3, dt, SolverOpts(lin=GmresOpts(m=20, rtol=1e-8), yhist=hp))
        sw = disc.row_step(Uw, 3, dt, SolverOpts(lin=GmresOpts(m=20, rtol=1e-8), yhist=hw, warm=warm))
        assert sp["status"] == 0 and sw["status"] == 0
        it_p += sp["gmres_iters"]
        it_w += sw["gmres_iters"]
        used += sw["warm_used"]
        rej += sw["warm_rejected"]
    print(f"GMRES iterations over 6 ROW3 steps: plain {it_p}, learned warm start {it_w} "
          f"(guesses used {used}, rejected {rej})", flush=True)
    assert it_w <= 1.05 * it_p
    assert rel(to_np(Uw), to_np(Up)) <= 1e-7


def _train(disc, logs, rng, steps=400):
    from paper_1904_04825_amd import MlpTrainer, WarmStart
    trainers = []
    for i, lg in enumerate(logs.logs):
        tr = MlpTrainer(disc, n_hidden=256, seed=14 + i, lr=1e-3)
        tr.fit_stats(lg)
        losses = [tr.step(lg, torch.as_tensor(rng.choice(lg.count, 512, replace=False), dtype=torch.int32,
                                              device="cuda")) for _ in range(steps)]
        assert np.mean(losses[-20:]) < 0.5 * losses[0]
        trainers.append(tr)
    return WarmStart([t.net for t in trainers])


@pytest.mark.parametrize("kind", ["esdirk3", "bdf2"])
def test_ptc_learned_start(kind):
    """ESDIRK3 and BDF2: log the converged stage increments, train one network per
    implicit stage, then start PTC from the learned guess where its ||F|| is smaller.
    Same nonlinear tolerance (relative to the plain start's ||F||): the states agree
    with the plain run's within the tolerance, and PTC needs no more iterations."""
    from paper_1904_04825_amd import GmresOpts, SolverOpts, StageLog, StageLogs
    _, op, disc = setup(16, 16, 3, "rusanov", seed=2)
    U0 = to_gpu(vortex_state(op, 0.0))
    dt, nst = 0.1, (3 if kind == "esdirk3" else 1)
    rng = np.random.default_rng(41)
    logs = StageLogs([StageLog(disc, 6000, rng.choice(disc.nel, 200, replace=False)) for _ in range(nst)])
    yh = torch.zeros((2, disc.ndof), dtype=torch.float64, device="cuda")
    lin = GmresOpts(m=20, rtol=1e-1)

    def step(U, Um1, opts):
        if kind == "esdirk3":
            st = disc.esdirk_step(U, 3, dt, opts)
            return U, None, st
        Un1, st = disc.bdf2_step(Um1, U, dt, opts)
        return Un1, U, st

    U, Um1 = U0.clone(), None
    for n in range(24):
        for lg in logs.logs:
            lg.set_elems(rng.choice(disc.nel, 200, replace=False))
        U, Um1, st = step(U, Um1, SolverOpts(lin=lin, tol_nl=1e-8, log=logs, yhist=yh))
        assert st["status"] == 0
    assert all(lg.count == 24 * 200 for lg in logs.logs)
    warm = _train(disc, logs, rng)
    Up, Upm1, hp = U.clone(), (Um1.clone() if Um1 is not None else None), yh.clone()
    Uw, Uwm1, hw = U.clone(), (Um1.clone() if Um1 is not None else None), yh.clone()
    ptc_p = ptc_w = used = 0
    for n in range(6):
        Up, Upm1, sp = step(Up, Upm1, SolverOpts(lin=lin, tol_nl=1e-8, yhist=hp))
        Uw, Uwm1, sw = step(Uw, Uwm1, SolverOpts(lin=lin, tol_nl=1e-8, yhist=hw, warm=warm))
        assert sp["status"] == 0 and sw["status"] == 0
        ptc_p += sp["ptc_iters"]
        ptc_w += sw["ptc_iters"]
        used += sw["warm_used"]
        assert sw["warm_used"] + sw["warm_rejected"] == nst
    print(f"{kind}: PTC iterations over 6 steps: plain {ptc_p}, learned start {ptc_w} (guesses used {used})",
          flush=True)
    assert used >= 3
    assert ptc_w <= ptc_p
    assert rel(to_np(Uw), to_np(Up)) <= 1e-6
