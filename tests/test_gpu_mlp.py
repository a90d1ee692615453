"""GPU parity of the learned proposal path against the FP64 oracle:
resampling, training samples, the network's forward pass, gradients and
Adam step, and the seeding draws; training is deterministic and lowers the
loss."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from paper_1208_4830_amd import inputs

pytestmark = pytest.mark.gpu

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def canon(p):
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k in NAMES])


def uncanon(v):
    out, o = {}, 0
    shapes = {"W1": (256, 512), "b1": (512,), "W2": (512, 512), "b2": (512,),
              "W3": (512, 120), "b3": (120,)}
    for k in NAMES:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(v[o:o + n], np.float64).reshape(shapes[k])
        o += n
    return out


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    t = torch.from_numpy(np.asarray(a, np.float32).copy()).to(torch.bfloat16)
    return t.to(torch.float64).numpy()


def gpu_params(p):
    """The values the network computes with: BF16 weights, FP32 biases."""
    q = {}
    for k in NAMES:
        v = np.asarray(p[k], np.float32).astype(np.float64)
        q[k] = bf16(v) if k.startswith("W") else v
    return q


def make_lcs(hip, lengths, seed, special=True):
    """CSR lightcurves with uniform cadence, random fluxes and weights."""
    rng = np.random.default_rng(seed)
    ts, ys, ws = [], [], []
    for k, L in enumerate(lengths):
        t = np.sort(rng.uniform(-50, 50, L))
        y = 1.0 + 0.2 * rng.random(L)
        w = rng.uniform(0.5, 2.0, L)
        ts.append(t), ys.append(y), ws.append(w)
    if special:
        # epochs crowded into the first bins plus one at the end, some with
        # zero weight; a lightcurve with no weight at all; a constant one
        t = np.concatenate([np.linspace(0, 0.3, 40), [100.0]])
        w = np.ones(41)
        w[::3] = 0.0
        ts.append(t), ys.append(np.cos(t)), ws.append(w)
        ts.append(np.linspace(0, 1, 9)), ys.append(np.ones(9)), ws.append(np.zeros(9))
        ts.append(np.linspace(0, 1, 33)), ys.append(np.full(33, 2.5)), ws.append(np.ones(33))
    off = np.zeros(len(ts) + 1, np.int64)
    off[1:] = np.cumsum([len(t) for t in ts])
    cat = [np.concatenate(a) if len(a) else np.zeros(0) for a in (ts, ys, ws)]
    dev = lambda a, dt=torch.float64: torch.tensor(a, dtype=dt, device="cuda")
    lcs = hip.Lightcurves(dev(off, torch.int64), dev(cat[0]), dev(cat[1]), dev(cat[2]))
    return lcs, off, cat


def test_resample_matches_oracle(hip):
    # empty, single-epoch and two-epoch lightcurves, sizes across many bins
    lengths = [0, 1, 2, 17, 255, 256, 257, 1000, 4999]
    lcs, off, (t, y, w) = make_lcs(hip, lengths, seed=3)
    xb, xf = hip.sblm_resample(lcs, want_f32=True, want_bf16=True)
    torch.cuda.synchronize()
    xf = xf.cpu().numpy().astype(np.float64)
    for k in range(len(off) - 1):
        sl = slice(off[k], off[k + 1])
        ref = M.resample(t[sl], y[sl], w[sl])
        err = np.abs(xf[k] - ref)
        assert np.all(err <= 1.2e-7 * np.abs(ref) + 1e-30), (k, err.max())
    # the BF16 output is the round-to-nearest-even of the FP32 one
    assert torch.equal(xb.cpu(), torch.from_numpy(xf.astype(np.float32)).to(torch.bfloat16))


def test_training_samples_match_oracle(hip):
    seed, first, n = 1234, 50, 12
    xb, xf, y = hip.mlp_make_data(seed, first, n, want_f32=True)
    torch.cuda.synchronize()
    xf, y = xf.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)
    for i in range(n):
        x_ref, y_ref = M.make_sample(seed, first + i)
        assert np.max(np.abs(xf[i] - x_ref)) < 1e-6, (i, np.max(np.abs(xf[i] - x_ref)))
        assert np.allclose(y[i], y_ref, rtol=2e-7, atol=1e-7), i
    # sample s depends only on (seed, s): a shifted range reproduces the rows
    xb2, _, y2 = hip.mlp_make_data(seed, first + 5, 4)
    assert torch.equal(xb2, xb[5:9]) and np.array_equal(y2.cpu().numpy(), y[5:9].astype(np.float32))


@pytest.mark.parametrize("rows", [192, 150])
def test_forward_matches_oracle(hip, rows):
    rng = np.random.default_rng(7)
    p = M.init_params(rng, scale_out=0.3)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(scale=0.1, size=p[k].shape)
    net = hip.MLP(batch_max=128, seed=1)  # rows span two chunks
    net.set_params(canon(p).astype(np.float32))
    x = bf16(rng.normal(size=(rows, 256)))
    out = net.forward(torch.tensor(x, dtype=torch.bfloat16, device="cuda"))
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    assert np.all(got[:, 120:] == 0)
    q = gpu_params(p)
    ref, _ = M.forward(q, x)
    rel = np.linalg.norm(got[:, :120] - ref) / np.linalg.norm(ref)
    # the kernels round the hidden activations to BF16; with that rounding
    # emulated only the FP32 accumulation order differs
    h1 = bf16(np.maximum(x @ q["W1"] + q["b1"], 0))
    h2 = bf16(np.maximum(h1 @ q["W2"] + q["b2"], 0))
    emu = h2 @ q["W3"] + q["b3"]
    scale = np.abs(h2) @ np.abs(q["W3"]) + np.abs(q["b3"])
    e_emu = np.abs(got[:, :120] - emu) / scale
    print(f"forward rows={rows}: rel vs FP64 {rel:.2e}, emulated max {e_emu.max():.2e}, "
          f"median {np.median(e_emu):.2e}")
    assert rel < 1e-2
    assert np.median(e_emu) < 1e-5 and e_emu.max() < 1e-2
    net.close()


def f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def test_gradients_match_oracle(hip):
    rng = np.random.default_rng(8)
    p = M.init_params(rng, scale_out=0.3)
    net = hip.MLP(batch_max=256, seed=1)
    net.set_params(canon(p).astype(np.float32))
    x = bf16(rng.normal(size=(256, 256)))
    y = rng.uniform(0, 1, (256, 7)).astype(np.float32)
    loss = net.loss_grad(torch.tensor(x, dtype=torch.bfloat16, device="cuda"),
                         torch.tensor(y, device="cuda"))
    g = uncanon(net.grad())
    L_ref, g_ref = M.loss_and_grad(gpu_params(p), x, y.astype(np.float64))
    L = float(loss.cpu())
    print(f"loss gpu {L:.6f} oracle {L_ref:.6f}")
    assert abs(L - L_ref) <= 1e-2 * abs(L_ref)
    # against FP64 backpropagation of the same network, tensor by tensor
    for k in NAMES:
        a, b = g[k].ravel(), g_ref[k].ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        print(f"  {k}: rel {rel:.2e} cos {cos:.6f}")
        assert rel < 3e-2 and cos > 0.999, k
    net.close()


def test_gradients_element_wise(hip):
    # Element by element against the oracle's backpropagation with the
    # kernels' roundings emulated: hidden activations BF16, output and output
    # gradient FP32 (the likelihood's gradient from the oracle), BF16 copies
    # of the output gradient and of the hidden-layer gradients as the
    # operands of the products; then only the FP32 accumulation order (and a
    # rare BF16 rounding decided the other way by it) differs.  Each entry's
    # error is scaled by the sum of the magnitudes of its terms, the
    # hidden-layer gradients taken at the magnitude of their own terms (where
    # they cancel to near zero, their rounding is relative to those terms).
    # Output weights of scale 0.05 give a loss of ~14, where the mixture's
    # posterior weights are not decided by the last bits of the FP32 outputs
    # (at scale 0.3 the loss is ~10^6 and one rounding of an output moves a
    # posterior weight by several per cent).
    rng = np.random.default_rng(18)
    p = M.init_params(rng, scale_out=0.05)
    net = hip.MLP(batch_max=256, seed=1)
    net.set_params(canon(p).astype(np.float32))
    x = bf16(rng.normal(size=(256, 256)))
    y = rng.uniform(0, 1, (256, 7)).astype(np.float32)
    loss = net.loss_grad(torch.tensor(x, dtype=torch.bfloat16, device="cuda"),
                         torch.tensor(y, device="cuda"))
    g = uncanon(net.grad())
    L = float(loss.cpu())
    q = gpu_params(p)
    h1 = bf16(np.maximum(x @ q["W1"] + q["b1"], 0))
    h2 = bf16(np.maximum(h1 @ q["W2"] + q["b2"], 0))
    o = f32(h2 @ q["W3"] + q["b3"])
    L_emu, dO = M.nll(o, y.astype(np.float64))
    print(f"loss gpu {L:.6f} emulated {L_emu:.6f}")
    assert abs(L - L_emu) <= 1e-5 * abs(L_emu)
    dOf = f32(dO)
    dOb = bf16(dOf)
    dZ2f = f32((dOb @ q["W3"].T) * (h2 > 0))
    dZ2b = bf16(dZ2f)
    dZ1f = f32((dZ2b @ q["W2"].T) * (h1 > 0))
    dZ1b = bf16(dZ1f)
    s2 = (np.abs(dOb) @ np.abs(q["W3"]).T) * (h2 > 0)   # magnitude of dZ2's terms
    s1 = (s2 @ np.abs(q["W2"]).T) * (h1 > 0)             # ... of dZ1's terms
    emu = {"W3": (h2.T @ dOb, np.abs(h2).T @ np.abs(dOb)),
           "W2": (h1.T @ dZ2b, np.abs(h1).T @ s2),
           "W1": (x.T @ dZ1b, np.abs(x).T @ s1),
           "b3": (dOf.sum(0), np.abs(dOf).sum(0)),
           "b2": (dZ2f.sum(0), s2.sum(0)),
           "b1": (dZ1f.sum(0), s1.sum(0))}
    for k in NAMES:
        ref, scale = emu[k]
        e = np.abs(g[k] - ref) / np.maximum(scale, 1e-6 * scale.max())
        print(f"  {k} element-wise vs emulated: median {np.median(e):.2e} "
              f"p99.9 {np.quantile(e, 0.999):.2e} max {e.max():.2e}")
    # One BF16 operand rounded the other way (a hidden activation, or an
    # output-gradient copy) moves its term by at most 2^-8 of its magnitude:
    # a flipped activation touches a whole row of its weight gradient, so
    # the 99.9th percentile may reach 2^-8, and no entry may pass 2.5 such
    # steps.  A wrong entry (a mis-indexed column, a lost slice of a split
    # sum) errs by O(1) of its scale.
    for k in NAMES:
        ref, scale = emu[k]
        e = np.abs(g[k] - ref) / np.maximum(scale, 1e-6 * scale.max())
        assert np.median(e) < 1e-5 and np.quantile(e, 0.999) < 2.0 ** -8 and e.max() < 1e-2, k
    net.close()


def test_adam_steps_match_oracle(hip):
    rng = np.random.default_rng(9)
    p = {"w": (rng.normal(size=455800) * 0.05).astype(np.float32).astype(np.float64)}
    net = hip.MLP(batch_max=64, seed=1)
    net.set_params(p["w"].astype(np.float32))
    st = {}
    for t, lr in ((1, 1e-3), (2, 5e-4), (3, 2e-3)):
        g = (rng.normal(size=455800) * 10.0 ** rng.uniform(-9, 0, 455800)).astype(np.float32)
        g[::1000] = 0.0
        net.set_grad(g)
        net.adam_step(lr)
        M.adam_step(p, {"w": g.astype(np.float64)}, st, lr=lr, t=t)
        got = net.get_params().astype(np.float64)
        err = np.abs(got - p["w"])
        assert np.all(err <= 2.4e-7 * np.abs(p["w"]) + 1e-9 * lr / 1e-3), (t, err.max())
    net.close()


def test_training_is_deterministic_and_lowers_the_loss(hip):
    xb, _, y = hip.mlp_make_data(3, 0, 8192)
    nets = [hip.MLP(batch_max=512, seed=5) for _ in range(2)]
    curves = [n.train(xb, y, batch=512, epochs=3, lr0=1e-3, lr1=1e-4) for n in nets]
    torch.cuda.synchronize()
    c = curves[0].cpu().numpy()
    print(f"training loss: first {c[:4].mean():.3f} last {c[-4:].mean():.3f}")
    assert np.all(np.isfinite(c)) and c[-4:].mean() < c[:4].mean() - 1.0
    assert torch.equal(curves[0], curves[1])
    assert np.array_equal(nets[0].get_params(), nets[1].get_params())
    for n in nets:
        n.close()


def test_training_graph_equals_stepping_through_the_api(hip):
    # mlp_train replays one captured step (batch gather, forward, likelihood,
    # backward, Adam with the split-K sums, step advance); it must give the
    # parameters and losses of the same steps taken one call at a time
    # (mlp_loss_grad + mlp_adam_step with the cosine learning rate), bit for
    # bit, and continue the step count (Adam's bias correction) across calls
    xb, _, y = hip.mlp_make_data(5, 0, 1024)
    a, b = hip.MLP(batch_max=256, seed=9), hip.MLP(batch_max=256, seed=9)
    f32 = lambda v: float(np.float32(v))
    lr0, lr1 = f32(1e-3), f32(1e-4)

    def steps_by_hand(batch, epochs):
        per = 1024 // batch
        total = per * epochs
        out = []
        for k in range(total):
            r0 = (k % per) * batch
            fr = k / (total - 1) if total > 1 else 0.0
            lr = f32(lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * fr)))
            out.append(b.loss_grad(xb[r0:r0 + batch], y[r0:r0 + batch]).item())
            b.adam_step(lr)
        return np.array(out, np.float32)

    for batch, epochs in ((256, 2), (256, 1), (128, 1)):  # split-K 2; again; new graph
        la = a.train(xb, y, batch=batch, epochs=epochs, lr0=lr0, lr1=lr1).cpu().numpy()
        lb = steps_by_hand(batch, epochs)
        torch.cuda.synchronize()
        assert np.array_equal(la, lb), (batch, epochs)
        assert np.array_equal(a.get_params(), b.get_params()), (batch, epochs)
        assert np.array_equal(a.grad(), b.grad()), (batch, epochs)
    a.close()
    b.close()


def test_seeding_matches_oracle(hip):
    lengths = [40, 0, 300, 1, 1200]
    lcs, off, (t, y, w) = make_lcs(hip, lengths, seed=4, special=False)
    cfg = hip.ea_default_config()
    cfg.pop = 16
    st = hip.EAState(cfg, lcs, 77)
    P0 = st.view("P").clone()
    rng = np.random.default_rng(5)
    out = np.zeros((len(lengths), 128), np.float32)
    out[:, :8] = rng.normal(size=(len(lengths), 8))
    out[:, 8:64] = rng.uniform(-0.2, 1.2, (len(lengths), 56))
    out[:, 64:120] = rng.uniform(-4, -0.5, (len(lengths), 56))
    st.seed(torch.tensor(out, device="cuda"), 9)
    torch.cuda.synchronize()
    P = st.view("P").cpu().numpy()
    P0 = P0.cpu().numpy()
    lo, hi = np.array(cfg.lo[:]), np.array(cfg.hi[:])
    for k, L in enumerate(lengths):
        cols = k * 16 + np.arange(16)
        if L == 0:
            assert np.array_equal(P[:, cols], P0[:, cols])
            continue
        tf = t[off[k]]
        span = t[off[k + 1] - 1] - tf
        ref = M.seed_rows(out[k].astype(np.float64), tf, span, lo, hi, 77, k, 9)
        assert np.allclose(P[:, cols[:9]].T, ref, rtol=0, atol=1e-12), k
        assert np.array_equal(P[:, cols[9:]], P0[:, cols[9:]])
    st.close()


def test_window_seeding_matches_oracle(hip):
    # the ablation of the learned form: rows from the observation window
    # alone (t0 mid-span, tE a quarter of the span, the rest uniform)
    lengths = [40, 0, 300, 1, 1200]
    lcs, off, (t, y, w) = make_lcs(hip, lengths, seed=14, special=False)
    cfg = hip.ea_default_config()
    cfg.pop = 16
    st = hip.EAState(cfg, lcs, 78)
    P0 = st.view("P").clone().cpu().numpy()
    st.seed_window(7)
    torch.cuda.synchronize()
    P = st.view("P").cpu().numpy()
    lo, hi = np.array(cfg.lo[:]), np.array(cfg.hi[:])
    for k, L in enumerate(lengths):
        cols = k * 16 + np.arange(16)
        if L == 0:
            assert np.array_equal(P[:, cols], P0[:, cols])
            continue
        tf = t[off[k]]
        span = t[off[k + 1] - 1] - tf
        ref = M.seed_rows(None, tf, span, lo, hi, 78, k, 7, window_only=True)
        assert np.allclose(P[:, cols[:7]].T, ref, rtol=0, atol=1e-12), k
        assert np.array_equal(P[:, cols[7:]], P0[:, cols[7:]])
        # every seeded row puts t0 at mid-span and tE at a quarter of it
        th = lo[:, None] + (hi - lo)[:, None] * P[:, cols[:7]]
        te = np.clip(span / 4, lo[4], hi[4])
        t0 = np.clip(tf + span / 2, lo[5], hi[5])
        assert np.allclose(th[4], te, atol=1e-9 * (hi[4] - lo[4]))
        assert np.allclose(th[5], t0, atol=1e-9 * (hi[5] - lo[5]))
    st.close()


def test_restarts_reseed_attached_proposals(hip):
    from oracle import oracle as O
    lengths = [60, 200, 0, 90]
    lcs, off, (t, y, w) = make_lcs(hip, lengths, seed=6, special=False)
    cfg = hip.ea_default_config()
    cfg.pop = 16
    cfg.stag_window, cfg.restart_after, cfg.stag_frac = 1, 1, 0.99  # restart often
    seed = 31
    st = hip.EAState(cfg, lcs, seed)
    rng = np.random.default_rng(6)
    out = np.zeros((len(lengths), 128), np.float32)
    out[:, :8] = rng.normal(size=(len(lengths), 8))
    out[:, 8:64] = rng.uniform(0, 1, (len(lengths), 56))
    out[:, 64:120] = rng.uniform(-3, -1, (len(lengths), 56))
    st.seed(torch.tensor(out, device="cuda"), 5, at_restarts=True)
    lo, hi = np.array(cfg.lo[:]), np.array(cfg.hi[:])
    prev = [s.n_restarts for s in st.summary()]
    checked = 0
    for _ in range(12):
        st.evaluate()
        st.generation(st.view("chi2"), st.view("Fs"), st.view("Fb"))
        summ = st.summary()
        P = st.view("P").cpu().numpy()
        for k, L in enumerate(lengths):
            if L == 0 or summ[k].n_restarts == prev[k]:
                continue
            g = summ[k].gen_restart
            cols = k * 16 + np.arange(16)
            tf, span = t[off[k]], t[off[k + 1] - 1] - t[off[k]]
            ref = M.seed_rows(out[k].astype(np.float64), tf, span, lo, hi, seed, k, 5, gen=g)
            assert np.allclose(P[:, cols[:5]].T, ref, rtol=0, atol=1e-12), (k, g)
            # the other rows are the fresh population of Sec. A.1 (antithetic pairs)
            for r in range(5, 16):
                i = r if r < 8 else r - 8
                u = np.array([O.u01(O.draw(seed, k, g, 1, i, j)) for j in range(6)])
                assert np.array_equal(P[:, cols[r]], u if r < 8 else 1.0 - u), (k, g, r)
            checked += 1
        prev = [s.n_restarts for s in summ]
    assert checked >= 3
    # detaching: a later restart draws the plain population again
    st.seed(torch.tensor(out, device="cuda"), 0)
    st.close()


def test_trained_network_improves_the_ea(hip):
    # a network trained on generated lightcurves seeds half of the population
    # at the start and at every restart; against the plain EA on the same
    # ragged lightcurves, EA seed and generation count
    xb, _, yt = hip.mlp_make_data(11, 0, 1 << 18)
    net = hip.MLP(batch_max=1024, seed=2)
    net.train(xb, yt, batch=1024, epochs=4, lr0=2e-3, lr1=1e-5)
    wl = inputs.ragged_workload(21, 256)
    t = torch.tensor(wl.t, device="cuda")
    A = torch.empty_like(t)
    for k in range(wl.n_lc):
        a, b = int(wl.off[k]), int(wl.off[k + 1])
        A[a:b] = hip.sblm_magnify(torch.tensor(wl.theta[:, k:k + 1].copy(), device="cuda"),
                                  t[a:b].contiguous())[0]
    L = np.diff(wl.off)
    F = np.repeat(wl.Fs, L) * A.cpu().numpy() + np.repeat(wl.Fb, L)
    sig = wl.sfrac * F
    lcs = hip.Lightcurves(torch.tensor(wl.off, device="cuda"), t,
                          torch.tensor(F + sig * wl.noise, device="cuda"),
                          torch.tensor(1.0 / sig ** 2, device="cuda"))
    c_true = hip.sblm_chi2(lcs, torch.tensor(wl.theta.copy(), device="cuda"), 1)[0].cpu().numpy()
    xr, _ = hip.sblm_resample(lcs)
    out = net.forward(xr)
    success = {}
    for form in ("plain", "window", "learned"):
        cfg = hip.ea_default_config()
        cfg.pop = 128
        st = hip.EAState(cfg, lcs, 7)
        if form == "learned":
            st.seed(out, 64, at_restarts=True)
        elif form == "window":  # the ablation: what the window alone gives
            st.seed_window(64, at_restarts=True)
        st.fit(150)
        best = np.array([s.best_chi2 for s in st.summary()])
        success[form] = float(np.mean(best <= c_true + 10.0))
        st.close()
    print(f"success after 150 generations: {success}")
    # the windows are random (t0 + tE (-3..-2) to t0 + tE (2..3)), so the
    # gain is what the network reads from the lightcurve's shape
    assert success["learned"] >= success["plain"] + 0.05
    assert success["learned"] >= success["window"] + 0.03
    net.close()
