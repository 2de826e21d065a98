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


@pytest.mark.parametrize("P", [2, 3, 4])
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


def _unflatten(flat, p0):
    g, o = {}, 0
    for name in ("1", "2", "3"):
        w = p0["W" + name]
        g["W" + name] = flat[o:o + w.size].reshape(w.shape)
        o += w.size
        g["b" + name] = flat[o:o + w.shape[0]]
        o += w.shape[0]
    return g


# P3: 256 -> 256 -> 256 -> 64; P4: 400 -> 256 -> 256 -> 100 (n_out not a multiple of 16)
@pytest.mark.parametrize("P", [3, 4])
def test_mlp_stats_gradients_and_adam(P):
    disc, tr = _trainer(P)
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
    g_gpu = _unflatten(tr.grad.cpu().numpy().astype(np.float64), p0)
    for k in g_or:
        print(f"P={P} {k} gradient rel err {rel(g_gpu[k], g_or[k]):.2e}", flush=True)
        assert rel(g_gpu[k], g_or[k]) <= 1e-3, k
    # one Adam step from the device gradients
    tr.step(lg, torch.as_tensor(idx, dtype=torch.int32, device="cuda"), lr=1e-3)
    p1 = _params_from_master(tr)
    g_used = _unflatten(tr.grad.cpu().numpy().astype(np.float64), p0)
    p_or = omlp.adam_step({k: v.copy() for k, v in p0.items()}, g_used, {}, lr=1e-3)
    for k in p_or:
        assert np.allclose(p1[k], p_or[k], rtol=1e-5, atol=1e-6), k


# fr_mlp_infer against the oracle's features -> forward -> decode, every element of the mesh
@pytest.mark.parametrize("P", [3, 4])
def test_mlp_infer_parity(P):
    disc, tr = _trainer(P)
    lg, _ = _synthetic_log(disc, 512, seed=7)
    tr.fit_stats(lg)
    _, op, _ = setup(6, 5, P, "rusanov")
    U = vortex_state(op)
    R = op.residual(U)
    dt = 0.1
    Y1 = fi.random_vector(U.shape, seed=31, scale=0.05 * dt)
    Y2 = fi.random_vector(U.shape, seed=32, scale=0.05 * dt)
    norm = tr.net.norm.cpu().numpy().astype(np.float64).reshape(20, 2)
    stats_in = [[tuple(norm[4 * f + v]) for v in range(4)] for f in range(4)]
    stats_out = [tuple(norm[16 + v]) for v in range(4)]
    p = _params_from_master(tr)
    for y1, y2 in ((Y1, Y2), (None, None)):
        x0 = to_np(tr.net.infer(to_gpu(U), to_gpu(R), None if y1 is None else to_gpu(y1),
                                None if y2 is None else to_gpu(y2), dt))
        z = np.zeros_like(U)
        X = omlp.features(U, R, z if y1 is None else y1, z if y2 is None else y2, dt, np.arange(op.nel), stats_in)
        yo, _ = omlp.forward(p, X, emulate_bf16=True)
        xo = omlp.decode(yo, stats_out, dt, disc.np_)
        print(f"P={P} infer ({'with' if y1 is not None else 'without'} previous increments): "
              f"rel err {rel(x0, xo):.2e}", flush=True)
        assert rel(x0, xo) <= 1e-3


def test_stage_log_rows_match_oracle():
    """The samples a ROW3 step logs: per element, float32 of q^n, R(q^n), Y_{i-1}/dt,
    Y_{i-2}/dt (the previous step's increments for the first stages) and the converged
    Y_i/dt, for the logged elements in the order given, against the oracle's step."""
    from oracle import integrators as I
    from oracle.tableaux import ROW
    from paper_1904_04825_amd import GmresOpts, SolverOpts, StageLog, StageLogs
    _, op, disc = setup(7, 5, 3, "rusanov", seed=8)
    U = vortex_state(op, 0.0)
    dt = 0.1
    hist = np.stack([fi.random_vector(U.shape, seed=41, scale=1e-3), fi.random_vector(U.shape, seed=42, scale=1e-3)])
    elems = np.random.default_rng(3).permutation(op.nel)[:20]
    logs = StageLogs([StageLog(disc, 20, elems) for _ in range(4)])
    yh = torch.as_tensor(hist.reshape(2, -1), device="cuda").contiguous()
    st = disc.row_step(to_gpu(U), 3, dt, SolverOpts(lin=GmresOpts(m=20, rtol=1e-10), log=logs, yhist=yh))
    assert st["status"] == 0 and all(lg.count == 20 for lg in logs.logs)
    _, so = I.row_step(op, ROW["ROW3"], dt, U, I.LinOpts(m=20, rtol=1e-10))
    Y = so.stage_increments
    R = op.residual(U)
    prev = [hist[1], hist[0]]          # newest first
    Np = disc.np_
    for i, lg in enumerate(logs.logs):
        Y1 = Y[i - 1] if i >= 1 else prev[0]
        Y2 = Y[i - 2] if i >= 2 else (prev[0] if i == 1 else prev[1])
        rows = lg.samples.cpu().numpy().astype(np.float64)
        for f, (a, tol) in enumerate(((U, 0.0), (R, 1e-6), (Y1 / dt, 1e-6), (Y2 / dt, 1e-6))):
            ref = np.concatenate([a[v][elems] for v in range(4)], axis=1).astype(np.float32).astype(np.float64)
            got = rows[:, f * 4 * Np:(f + 1) * 4 * Np]
            if tol == 0.0:
                assert np.array_equal(got, ref), (i, f)
            else:
                assert rel(got, ref) <= tol, (i, f, rel(got, ref))
        tgt = np.concatenate([(Y[i] / dt)[v][elems] for v in range(4)], axis=1)
        err = rel(rows[:, 16 * Np:], tgt)
        print(f"stage {i}: logged target rel err {err:.2e}", flush=True)
        assert err <= 1e-6


def test_row3_learned_warm_start():
    """Log the stage solves of 24 ROW3 steps of the vortex on a 32x32 perturbed P3 mesh
    (every element: 24,576 samples per stage), train one network per stage on the GPU,
    then run 6 later steps (held out: states the networks never saw) with and without
    the learned guess.  Same tolerance, relative to the zero guess's residual: the
    learned guess must save at least 7% of the GMRES iterations (measured: 9.9%)."""
    from paper_1904_04825_amd import GmresOpts, MlpTrainer, SolverOpts, StageLog, StageLogs, WarmStart
    _, op, disc = setup(32, 32, 3, "rusanov", seed=2)
    U0 = to_gpu(vortex_state(op, 0.0))
    dt, S, nlog = 0.1, 4, 24
    rng = np.random.default_rng(40)
    logs = StageLogs([StageLog(disc, nlog * disc.nel, np.arange(disc.nel)) for _ in range(S)])
    yhist = torch.zeros((2, disc.ndof), dtype=torch.float64, device="cuda")
    U = U0.clone()
    opts = SolverOpts(lin=GmresOpts(m=20, rtol=1e-8), log=logs, yhist=yhist)
    for n in range(nlog):
        st = disc.row_step(U, 3, dt, opts)
        assert st["status"] == 0
    assert all(lg.count == nlog * disc.nel for lg in logs.logs)
    trainers = []
    steps = 1500
    for i, lg in enumerate(logs.logs):
        tr = MlpTrainer(disc, n_hidden=256, seed=4 + i, lr=1e-3)
        tr.fit_stats(lg)
        losses = []
        for it in range(steps):
            idx = torch.as_tensor(rng.choice(lg.count, 1024, replace=False), dtype=torch.int32, device="cuda")
            losses.append(tr.step(lg, idx, lr=1e-3 * 0.5 * (1 + np.cos(np.pi * it / steps))))
        print(f"stage {i}: loss {losses[0]:.3e} -> {np.mean(losses[-20:]):.3e}", flush=True)
        assert np.mean(losses[-20:]) < 0.1 * losses[0]
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
    print(f"GMRES iterations over 6 held-out ROW3 steps: plain {it_p}, learned warm start {it_w} "
          f"(guesses used {used}, rejected {rej})", flush=True)
    assert used == 6 * S
    assert it_w <= 0.93 * it_p
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
    ptc_p = ptc_w = used = gm_p = gm_w = 0
    for n in range(6):
        Up, Upm1, sp = step(Up, Upm1, SolverOpts(lin=lin, tol_nl=1e-8, yhist=hp))
        Uw, Uwm1, sw = step(Uw, Uwm1, SolverOpts(lin=lin, tol_nl=1e-8, yhist=hw, warm=warm))
        assert sp["status"] == 0 and sw["status"] == 0
        ptc_p += sp["ptc_iters"]
        ptc_w += sw["ptc_iters"]
        gm_p += sp["gmres_iters"]
        gm_w += sw["gmres_iters"]
        used += sw["warm_used"]
        assert sw["warm_used"] + sw["warm_rejected"] == nst
    print(f"{kind}: PTC iterations over 6 steps: plain {ptc_p}, learned start {ptc_w}; GMRES iterations plain "
          f"{gm_p}, learned {gm_w} (guesses used {used})", flush=True)
    assert used >= 3
    assert ptc_w <= ptc_p
    assert rel(to_np(Uw), to_np(Up)) <= 1e-6


def test_group_training_matches_single():
    """fr_mlp_train_group: three P4 networks (400 -> 256 -> 256 -> 100) trained together on
    their own logs end bitwise where MlpTrainer.fit leaves each one alone (same batches,
    same learning-rate schedule): master weights, Adam moments, bf16 weights, biases and
    the losses read along the way.  Batch 1024 takes the split-K weight-gradient path."""
    from paper_1904_04825_amd import MlpTrainer, fit_group
    _, op, disc = setup(6, 5, 4, "rusanov")
    logs = [_synthetic_log(disc, 3000, 20 + q)[0] for q in range(3)]
    steps, batch = 25, 1024
    single, group = [], []
    for q in range(3):
        a = MlpTrainer(disc, n_hidden=256, seed=30 + q)
        b = MlpTrainer(disc, n_hidden=256, seed=30 + q)
        for tr in (a, b):
            tr.fit_stats(logs[q])
        single.append((a, a.fit(logs[q], steps, batch, lr=2e-3, seed=50 + q, report_every=10)))
        group.append(b)
    out = fit_group(group, logs, steps, batch, lr=2e-3, seeds=[50, 51, 52], report_every=10)
    torch.cuda.synchronize()
    for q in range(3):
        a, la = single[q]
        b = group[q]
        assert [s for s, _ in la] == [s for s, _ in out[q]]
        assert [l for _, l in la] == [l for _, l in out[q]], (la, out[q])
        assert all(np.isfinite(l) for _, l in la)  # the synthetic targets are noise: no learning asserted
        for name in ("master", "m", "v"):
            assert torch.equal(getattr(a, name), getattr(b, name)), (q, name)
        assert torch.equal(a.net.w, b.net.w) and torch.equal(a.net.b, b.net.b), q
        assert a.c.t == b.c.t == steps
