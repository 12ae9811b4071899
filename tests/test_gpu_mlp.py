"""GPU parity of the learned first-floor selector (addition (4)) and of its
density statistics against the CPU FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import features as ofeat
from oracle import mlp as omlp
from paper_2607_26382_amd import selector as sel
from paper_2607_26382_amd import synth
from paper_2607_26382_amd import topoguard as tg
from paper_2607_26382_amd._lib import TopoguardError

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _oracle_params(seed):
    return omlp.init_params(seed)


def _std_inputs(B, seed):
    rng = np.random.default_rng(seed)
    std = np.array([1, 1, 0.2, 0.1, 0.05, 2, 0.3, 0.4])
    mean = np.array([-3, -4, 0.5, 0.25, 0.02, 8, 0.4, 5.0])
    X = rng.standard_normal((B, 8)) * std + mean
    return X, mean, std


def _grads_flat(grads):
    return np.concatenate([g.ravel() for g in grads])


@pytest.mark.parametrize("B", [1, 5, 64, 257, 3000])
def test_forward_matches_oracle(B):
    params = _oracle_params(1)
    X, mean, std = _std_inputs(B, 2)
    m = tg.MLP(params, mean, std, max_batch=64)
    logits = m.forward(torch.tensor(X, dtype=torch.float32, device=DEV)).cpu().numpy()
    Xf = X.astype(np.float32).astype(np.float64)
    ref, _ = omlp.forward([p.astype(np.float32).astype(np.float64) for p in params],
                          (Xf - mean.astype(np.float32)) / std.astype(np.float32))
    assert np.abs(logits - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    # argmax decisions agree wherever the oracle's margin exceeds the FP32 error
    srt = np.sort(ref, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-3
    assert np.array_equal(np.argmax(logits, 1)[clear], omlp.predict(
        [p.astype(np.float32).astype(np.float64) for p in params],
        (Xf - mean.astype(np.float32)) / std.astype(np.float32))[clear])


@pytest.mark.parametrize("B,seed", [(1, 0), (7, 1), (256, 2), (1000, 3)])
def test_gradients_match_oracle(B, seed):
    params = [p.astype(np.float32).astype(np.float64) for p in _oracle_params(seed)]
    X, mean, std = _std_inputs(B, 10 + seed)
    y = np.random.default_rng(20 + seed).integers(0, 4, B)
    m = tg.MLP(params, mean, std)
    xd = torch.tensor(X, dtype=torch.float32, device=DEV)
    yd = torch.tensor(y, dtype=torch.int32, device=DEV)
    loss, g = m.train_step(xd, yd, lr=0.0, want_grads=True)
    Xs = (X.astype(np.float32).astype(np.float64) - mean.astype(np.float32)) / std.astype(np.float32)
    ref_loss, ref_grads = omlp.loss_and_grads(params, Xs, y)
    assert abs(loss - ref_loss) <= 1e-5 * max(1.0, ref_loss)
    g = g.cpu().numpy().astype(np.float64)
    o = 0
    for rg in ref_grads:
        n = rg.size
        gg = g[o:o + n]
        o += n
        # FP32 vs FP64: within 1e-4 of the tensor's largest gradient
        assert np.abs(gg - rg.ravel()).max() <= 1e-4 * max(np.abs(rg).max(), 1e-6)
    assert o == tg.N_PARAMS
    # lr = 0 leaves the parameters untouched
    assert np.array_equal(m.get_params(), tg.MLP.flatten(params))


def test_adam_steps_match_oracle_update():
    params = [p.astype(np.float32).astype(np.float64) for p in _oracle_params(4)]
    X, mean, std = _std_inputs(300, 5)
    y = np.random.default_rng(6).integers(0, 4, 300)
    m = tg.MLP(params, mean, std)
    xd = torch.tensor(X, dtype=torch.float32, device=DEV)
    yd = torch.tensor(y, dtype=torch.int32, device=DEV)
    Xs = (X.astype(np.float32).astype(np.float64) - mean.astype(np.float32)) / std.astype(np.float32)
    ref = [p.copy() for p in params]
    state = {}
    robust = None
    lr, b1, b2 = 1e-2, 0.9, 0.999
    prev = m.get_params().astype(np.float64)
    for step in range(3):
        m.train_step(xd, yd, lr=lr)
        # the oracle's own gradient and Adam step on the same inputs
        _, rg = omlp.loss_and_grads(ref, Xs, y)
        if robust is None:
            # parameters whose gradient is well away from zero: the FP32 and
            # FP64 gradients share their sign and agree to ~1e-4 relative, so
            # Adam's normalized steps agree closely; elsewhere Adam's step
            # (at most ~lr per parameter and step) may differ in sign
            robust = np.concatenate([np.abs(g.ravel()) >= 1e-2 * np.abs(g).max() for g in rg])
        omlp.adam_step(ref, rg, state, lr=1e-2)
        got = m.get_params().astype(np.float64)
        want = tg.MLP.flatten(ref).astype(np.float64)
        assert np.abs(got - want)[robust].max() <= 2e-4 * (step + 1), step
        # every parameter: Adam's step m^/(sqrt(v^) + eps) is a weighted mean
        # of gradients over a weighted root mean square of the same
        # gradients, so by Cauchy-Schwarz |step| <= lr sqrt(sum_i w_i^2 / u_i)
        # with the bias-corrected weights w_i of the first moment and u_i of
        # the second (1.0 at t = 1, 1.004 at t = 3); a missing bias
        # correction or a swapped beta exceeds it
        t = step + 1
        w = np.array([b1 ** (t - i) * (1 - b1) / (1 - b1 ** t) for i in range(1, t + 1)])
        u = np.array([b2 ** (t - i) * (1 - b2) / (1 - b2 ** t) for i in range(1, t + 1)])
        bound = lr * np.sqrt(np.sum(w * w / u))
        ulp = float(np.spacing(np.float32(np.abs(got).max())))   # FP32 parameters
        assert np.abs(got - prev).max() <= bound * (1 + 1e-5) + 2 * ulp, step
        prev = got
    assert robust.mean() > 0.5


def test_training_is_deterministic_and_learns_a_rule():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((2048, 8)).astype(np.float32)
    # a label that the probe rule would produce from its two features
    y = ((X[:, 0] > 0.3) | ((X[:, 1] > -0.2) & (X[:, 1] - X[:, 0] > -0.5))).astype(np.int32) + \
        (X[:, 4] > 1.0).astype(np.int32)
    runs = []
    for _ in range(2):
        m = tg.MLP(sel.init_params(0), X.mean(0), X.std(0), max_batch=256)
        xd, yd = torch.tensor(X, device=DEV), torch.tensor(y, device=DEV)
        losses = []
        for ep in range(60):
            perm = torch.tensor(np.random.default_rng(ep).permutation(2048), device=DEV)
            for b0 in range(0, 2048, 256):
                ix = perm[b0:b0 + 256]
                losses.append(m.train_step(xd[ix], yd[ix], 3e-3))
        runs.append((m.get_params(), losses))
    assert np.array_equal(runs[0][0], runs[1][0])     # bitwise reproducible
    assert runs[0][1][-1] < 0.5 * runs[0][1][0]
    pred = np.argmax(m.forward(torch.tensor(X, device=DEV)).cpu().numpy(), axis=1)
    assert np.mean(pred == y) > 0.9


def test_mlp_invalid_arguments():
    m = tg.MLP()
    x = torch.zeros((2, 8), dtype=torch.float32, device=DEV)
    with pytest.raises(TopoguardError, match="not set"):
        m.forward(x)
    bad = sel.init_params(0)
    bad[3] = np.nan
    with pytest.raises(TopoguardError, match="finite"):
        m.set_params(bad)
    with pytest.raises(TopoguardError, match="> 0"):
        m.set_params(sel.init_params(0), np.zeros(8), np.zeros(8))


def _bar(nx, ny, nz, cut=None):
    rho = np.zeros((nz, ny, nx))
    rho[0, :, :] = 1.0            # bottom layer from the clamped face to the loaded edge
    if cut is not None:
        rho[:, :, cut] = 0.0
    return rho.ravel()


FEATURE_CASES = [
    ("blobs", (16, 8, 8)), ("uniform", (17, 9, 7)), ("struts", (32, 16, 16)), ("bar", (12, 6, 4)),
    ("cutbar", (12, 6, 4)), ("zeros", (8, 4, 4)), ("ones", (1, 1, 1)), ("severe", (64, 32, 32)),
    ("selector", (48, 24, 24)),
]


def _feature_field(kind, dims):
    if kind == "blobs":
        return synth.blobs(*dims, 3, blob=2, floor_frac=0.4)
    if kind == "uniform":
        return synth.uniform(*dims, 4)
    if kind == "struts":
        return synth.struts(*dims, 5, n_struts=6, background=0.0, sigma=(1.0, 2.0))
    if kind == "bar":
        return _bar(*dims)
    if kind == "cutbar":
        return _bar(*dims, cut=5)
    if kind == "zeros":
        return np.zeros(dims[0] * dims[1] * dims[2])
    if kind == "ones":
        return np.ones(1)
    if kind == "severe":
        return synth.severe(1000)[1]
    return synth.selector_state(6_000_001, dims)[1]


@pytest.mark.parametrize("kind,dims", FEATURE_CASES)
@pytest.mark.parametrize("rho0", [1e-9, 1e-3])
def test_density_features_match_oracle(kind, dims, rho0):
    rho = _feature_field(kind, dims)
    g = tg.Grid(*dims, max_restart=4, device=DEV)
    got = g.density_features(torch.tensor(rho, device=DEV), 3.0, rho0)
    ref = ofeat.density_stats(rho, *dims, 3.0, rho0)
    assert got[0] == ref[0]                      # exact count ratio
    assert abs(got[1] - ref[1]) <= 1e-14 * max(1.0, abs(ref[1]))
    assert got[2] == ref[2]                      # a stored value
    assert abs(got[3] - ref[3]) <= 1e-12 * max(1.0, abs(ref[3]))
    assert got[4] == ref[4]                      # exact count ratio (component labels are unique)
    assert abs(got[5] - ref[5]) <= 1e-15 * ref[5]
    if kind == "bar":
        assert got[4] == 1.0
    if kind == "cutbar":
        assert got[4] == 0.0


def _small_batch(n, dims=(16, 8, 8), seed0=50):
    grids = [tg.Grid(*dims, max_restart=100, device=DEV) for _ in range(n)]
    rhos = [torch.tensor(synth.blobs(*dims, seed0 + i, blob=2, floor_frac=0.5), device=DEV) for i in range(n)]
    f = torch.tensor(grids[0].edge_load(), device=DEV)
    return grids, rhos, [f] * n


def test_policy_with_mlp_selector_follows_prediction():
    """A network whose output layer is a constant picks that rung for every
    state; the ladder from there is the FIXED(k) ladder, attempt by attempt."""
    grids, rhos, fs = _small_batch(4)
    batch = tg.Batch(grids)
    solve = tg.solver_opts(prec=tg.F32)
    for k in range(4):
        p = sel.init_params(0)
        p[-4 - 256:-4] = 0.0                      # W3 = 0
        p[-4:] = 0.0
        p[-4 + k] = 1.0                           # b3 = e_k
        m = tg.MLP(p)
        _, rm = batch.select_floor(rhos, fs, tg.policy(selector=tg.SELECT_MLP, mlp=m, solve=solve))
        _, rf = batch.select_floor(rhos, fs, tg.policy(selector=tg.SELECT_FIXED, fixed_rung=k, solve=solve,
                                                       want_features=True))
        for a, b in zip(rm, rf):
            assert a["k0"] == k and b["k0"] == k
            assert a["rung"] == b["rung"] and a["attempts"] == b["attempts"]
            assert a["features"] == b["features"]   # same probe, same statistics


def test_policy_features_equal_density_features():
    grids, rhos, fs = _small_batch(3, seed0=70)
    batch = tg.Batch(grids)
    _, res = batch.select_floor(rhos, fs, tg.policy(want_features=True, solve=tg.solver_opts(prec=tg.F32)))
    for g, r, out in zip(grids, rhos, res):
        st = g.density_features(r, 3.0, 1e-9)
        assert np.allclose(out["features"][2:], np.float32(st), rtol=0, atol=0)
        assert out["features"][0] == pytest.approx(np.log10(out["r50"]), abs=1e-6)


def test_learned_selector_gain_online_and_exact_replay():
    """On held-out mixture states, the stored network's first rungs put more
    first attempts at the lowest admissible rung and spend fewer iterations
    than the two-feature rule; the online policies make exactly the attempts
    the offline replay predicts; every accepted solution passed the FP64
    residual guard (false acceptances: 0)."""
    mlp, _ = sel.load_model()
    dims = (32, 16, 16)
    seeds = list(range(6_100_000, 6_100_048))
    states = [synth.selector_state(s, dims) for s in seeds]
    grids = [tg.Grid(*dims, max_restart=100, device=DEV) for _ in seeds]
    batch = tg.Batch(grids)
    rhos = [torch.tensor(r, device=DEV) for _, r, _ in states]
    f = torch.tensor(grids[0].edge_load(), device=DEV)
    solve = tg.solver_opts(prec=tg.BF16X3MFMA)
    runs = {}
    for name, pol in (("rule", tg.policy(solve=solve)),
                      ("mlp", tg.policy(selector=tg.SELECT_MLP, mlp=mlp, solve=solve))):
        us, res = batch.select_floor(rhos, [f] * len(seeds), pol)
        runs[name] = (us, res)
    del batch
    labels = sel.label_states(seeds, dims, log=lambda *a, **k: None)
    summ = {}
    for name, (us, res) in runs.items():
        k0 = np.array([r["k0"] for r in res])
        rp = sel.replay(labels, k0)
        for i, r in enumerate(res):
            assert r["rung"] == rp["rung"][i] and len(r["attempts"]) == rp["attempts"][i], (name, i)
            assert r["iters_rejected"] == rp["iters_rejected"][i]
            if r["rung"] >= 0:
                # the FP64 guard's verdict (its parity with the oracle on
                # seeded vectors: test_gpu_parity.test_true_residual_parity)
                assert r["attempts"][-1]["accepted"] and r["attempts"][-1]["true_eta"] <= 1e-6, (name, i)
        summ[name] = sel.summarize(labels, k0)
    assert summ["mlp"]["first_at_lowest"] > summ["rule"]["first_at_lowest"]
    assert summ["mlp"]["total_iters_per_state"] < summ["rule"]["total_iters_per_state"]
    assert summ["mlp"]["certified"] == summ["rule"]["certified"] == int(np.count_nonzero(labels["label"] >= 0))
