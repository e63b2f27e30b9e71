"""GPU tests of the learned bucket classifier against the FP64 oracle.

Feature export: every candidate bucket of every round, compared per (signal,
round, bucket) with the oracle's features, labels and decisions.  Network:
forward probabilities and the cross-entropy gradient against the FP64 network
on the same BF16-rounded parameters and inputs.  Training on GPU-exported
features, then a learned recovery compared with the oracle using the same
trained parameters.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import classifier as C

pytestmark = pytest.mark.gpu


def _sfft():
    from paper_1606_07407_amd import sfft
    return sfft


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _c4_batch(B, k, seed_off=0):
    cfg = workloads.config("c4")
    sig = workloads.planted.uniform_sigma(cfg["seed"] + seed_off, B, 0.0, 1e-2)
    pb = workloads.planted_batch(cfg["seed"] + seed_off, B, cfg["d"], cfg["N"], k, cfg["mag"], sig)
    return cfg, pb


def _plan(cfg, k_max, B, **over):
    sfft = _sfft()
    kw = dict(d=cfg["d"], N=cfg["N"], k_max=k_max, d1=cfg["d1"], c=cfg["c"],
              p_min=cfg["p_min"], ladder_K=cfg["ladder_K"], tau=cfg["tau"], eta=cfg["eta"],
              precision=sfft.SFFT_FP32, robust=int(cfg["robust"]), verify=int(cfg["verify"]),
              verify_eta=cfg["verify_eta"] or 0.0, residual=int(cfg["residual"]))
    kw.update(over)
    return sfft.sfft_plan_create(sfft.Params(**kw), max_batch=B)


def _oracle_params(cfg, k, **over):
    kw = dict(d=cfg["d"], N=cfg["N"], k=int(k), d1=cfg["d1"], c=cfg["c"],
              ladder_K=cfg["ladder_K"], tau=cfg["tau"], eta=cfg["eta"], p_min=cfg["p_min"],
              robust=cfg["robust"], verify=cfg["verify"], verify_eta=cfg["verify_eta"])
    kw.update(over)
    return oracle.Params(**kw)


def _export(cfg, pb, cap=200000, **over):
    import torch
    sfft = _sfft()
    plan = _plan(cfg, int(pb.k.max()), pb.B, **over)
    out = sfft.alloc_outputs(plan, pb.B, export_cap=cap)
    sfft.sfft_recover(plan, sfft.DeviceBatch.from_planted(pb), out)
    torch.cuda.synchronize()
    n = int(out["feat_count"].item())
    assert n <= cap
    res = dict(feat=out["feat"][:n].cpu().numpy(), label=out["label"][:n].cpu().numpy(),
               meta=out["feat_meta"][:n].cpu().numpy(), out=sfft.outputs_to_host(out))
    plan.close()
    return res


def test_export_matches_oracle():
    cfg, pb = _c4_batch(3, 150)
    g = _export(cfg, pb)
    _say(f"[export] {len(g['label'])} records")
    gpu = {(int(m[0]), int(m[1]), int(m[2])): (f, int(l), int(m[3]))
           for f, l, m in zip(g["feat"], g["label"], g["meta"])}
    assert len(gpu) == len(g["label"])  # no duplicate (signal, round, bucket)
    n_ref = 0
    u = 2.0 ** -24
    for b in range(pb.B):
        w, a = pb.signal(b)
        col = []
        r = oracle.multiphaseshift(w, a, _oracle_params(cfg, pb.k[b]), sigma=float(pb.sigma[b]),
                                   seed=pb.seed, signal=b, collect=col)
        p_of = {t["i"]: t["p"] for t in r.trace}
        for (i, h, x, lab, acc, a_h) in col:
            key = (b, i, h)
            assert key in gpu, key
            f, gl, ga = gpu[key]
            assert gl == lab and ga == acc, (key, gl, lab, ga, acc)
            # FP32 spectra: F_0/p carries an absolute error of order
            # u log2(L) sqrt(sum |a|^2 / p); the ratios z carry that over |F_0|/p,
            # and the features (asinh of deviations / tau) that over tau.
            p = p_of[i]
            L = 1 << int(np.ceil(np.log2(2 * p - 1)))
            dz = 20 * u * np.log2(L) * np.sqrt(np.sum(np.abs(a) ** 2) / p) / a_h
            tol = 5e-3 + dz / cfg["tau"]
            assert np.abs(f - x).max() <= tol, (key, f, x, tol)
            n_ref += 1
    assert n_ref == len(gpu)


def test_export_entry_point_equals_recover_export():
    """sfft_export_bucket_features writes the same records as sfft_recover's optional
    export on the same batch (bit for bit; the order across signals may differ)."""
    import torch
    sfft = _sfft()
    cfg, pb = _c4_batch(4, 150)
    g = _export(cfg, pb)
    plan = _plan(cfg, int(pb.k.max()), pb.B)
    out = sfft.sfft_export_bucket_features(plan, sfft.DeviceBatch.from_planted(pb), 200000)
    torch.cuda.synchronize()
    n = int(out["feat_count"].item())
    plan.close()
    assert n == len(g["label"]) and n > 0
    f, lab, meta = (out["feat"][:n].cpu().numpy(), out["label"][:n].cpu().numpy(),
                    out["feat_meta"][:n].cpu().numpy())
    o1 = np.lexsort(meta[:, :3].T[::-1])
    o2 = np.lexsort(g["meta"][:, :3].T[::-1])
    assert np.array_equal(meta[o1], g["meta"][o2])
    assert np.array_equal(lab[o1], g["label"][o2])
    assert np.array_equal(f[o1], g["feat"][o2])
    # a too-small cap counts every record and writes only the first cap
    plan = _plan(cfg, int(pb.k.max()), pb.B)
    small = sfft.sfft_export_bucket_features(plan, sfft.DeviceBatch.from_planted(pb), 7)
    torch.cuda.synchronize()
    plan.close()
    assert int(small["feat_count"].item()) == n
    _say(f"[export entry] {n} records equal the recovery's export")


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    th = C.init_params(seed) + rng.normal(scale=0.05, size=C.N_PARAMS)
    return C.bf16_round(th)


def _to_bf16_tensor(theta):
    import torch
    return torch.tensor(theta, dtype=torch.float32).to(torch.bfloat16).cuda()


def test_mlp_forward_and_grad_match_oracle():
    import torch
    sfft = _sfft()
    theta = _rand_params(5)
    rng = np.random.default_rng(6)
    X = rng.normal(scale=2.0, size=(3000, 8)).astype(np.float32)
    y = rng.integers(0, 2, size=3000).astype(np.uint8)
    w = _to_bf16_tensor(theta)
    xt = torch.tensor(X, device="cuda")
    yt = torch.tensor(y, device="cuda")
    prob = sfft.sfft_mlp_forward(w, xt).cpu().numpy()
    Xb = C.bf16_round(X.astype(np.float64))
    ref = C.prob_single(theta, Xb)
    _say(f"[mlp] forward max err {np.abs(prob - ref).max():.2e}")
    assert np.abs(prob - ref).max() < 2e-5
    loss, grad = sfft.sfft_mlp_grad(w, xt, yt)
    rl, rg = C.loss_and_grad(theta, Xb, y)
    gl, gg = float(loss.item()), grad.cpu().numpy()
    err = np.abs(gg - rg).max() / np.abs(rg).max()
    _say(f"[mlp] loss {gl:.6f} vs {rl:.6f}; grad rel err {err:.2e}")
    assert abs(gl - rl) <= 1e-5 * max(1.0, abs(rl))
    assert err < 1e-4


def test_mlp_grad_is_deterministic_and_loss_finite():
    """The gradient's sums over rows are added in a fixed order: 20000 rows (157 tiles over
    64 work-groups) give bit-identical results on repeated calls.  With logits far apart
    (the output layer scaled up) the loss is logsumexp(z) - z[label] per row, finite and
    equal to that expression on the oracle network's logits."""
    import torch
    sfft = _sfft()
    theta = _rand_params(9)
    rng = np.random.default_rng(10)
    X = rng.normal(scale=2.0, size=(20000, 8)).astype(np.float32)
    y = rng.integers(0, 2, size=20000).astype(np.uint8)
    xt = torch.tensor(X, device="cuda")
    yt = torch.tensor(y, device="cuda")
    w = _to_bf16_tensor(theta)
    l1, g1 = sfft.sfft_mlp_grad(w, xt, yt)
    l2, g2 = sfft.sfft_mlp_grad(w, xt, yt)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)
    Xb = C.bf16_round(X.astype(np.float64))
    rl, rg = C.loss_and_grad(theta, Xb, y)
    err = np.abs(g1.cpu().numpy() - rg).max() / np.abs(rg).max()
    _say(f"[mlp] 20000 rows: loss {float(l1.item()):.6f} vs {rl:.6f}; grad rel err {err:.2e}")
    assert abs(float(l1.item()) - rl) <= 1e-5 * max(1.0, abs(rl)) and err < 1e-4
    # saturated logits: output weights x 2^12 (exact in BF16)
    big = theta.copy()
    o3 = C.N_PARAMS - (2 * 64 + 2)
    big[o3:] *= 4096.0
    lb, _ = sfft.sfft_mlp_grad(_to_bf16_tensor(big), xt, yt)
    z, _ = C.forward(big, Xb)
    zm = z.max(axis=1)
    ref = float(np.mean(zm + np.log(np.exp(z[:, 0] - zm) + np.exp(z[:, 1] - zm))
                        - z[np.arange(len(y)), y.astype(np.int64)]))
    _say(f"[mlp] saturated logits: loss {float(lb.item()):.6e} vs {ref:.6e} "
         f"(largest logit gap {np.abs(z[:, 0] - z[:, 1]).max():.3e})")
    assert np.abs(z[:, 0] - z[:, 1]).max() > 200.0   # exp(-gap) underflows FP32
    assert np.isfinite(float(lb.item())) and abs(float(lb.item()) - ref) <= 1e-4 * abs(ref)


def test_train_then_learned_recovery():
    import torch
    sfft = _sfft()
    cfg, pb = _c4_batch(48, 300)
    g = _export(cfg, pb)
    sig_of = g["meta"][:, 0]
    train = sig_of < 40
    X = torch.tensor(g["feat"][train], device="cuda")
    Y = torch.tensor(g["label"][train], device="cuda")
    w = _to_bf16_tensor(C.bf16_round(C.init_params(11)))
    hist = sfft.sfft_mlp_train(w, X, Y, epochs=30, batch=512, lr=3e-3, seed=7).cpu().numpy()
    _say(f"[train] {int(train.sum())} rows; loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    assert hist[-1] < 0.5 * hist[0]
    # held-out signals: learned decisions vs labels, and the plain test's decisions
    Xt = torch.tensor(g["feat"][~train], device="cuda")
    p = sfft.sfft_mlp_forward(w, Xt).cpu().numpy()
    lab = g["label"][~train]
    acc_mlp = float(np.mean((p > 0.5) == (lab == 1)))
    acc_plain = float(np.mean(g["meta"][~train, 3] == lab))
    _say(f"[train] held-out accuracy: learned {acc_mlp:.4f}, plain test {acc_plain:.4f}")
    assert acc_mlp >= 0.97
    # learned recovery on fresh signals equals the oracle with the same parameters
    theta = w.to(torch.float32).cpu().numpy().astype(np.float64)
    cfg2, pb2 = _c4_batch(3, 150, seed_off=77)
    plan = _plan(cfg2, 150, pb2.B, classifier=sfft.SFFT_CLS_MLP, mlp_weights=w,
                 mlp_threshold=0.5)
    out = sfft.outputs_to_host(sfft.sfft_recover(plan, sfft.DeviceBatch.from_planted(pb2)))
    torch.cuda.synchronize()
    for b in range(pb2.B):
        wv, a = pb2.signal(b)
        ref = oracle.multiphaseshift(wv, a, _oracle_params(cfg2, 150, classifier="mlp",
                                                           mlp_params=theta, mlp_threshold=0.5),
                                     sigma=float(pb2.sigma[b]), seed=pb2.seed, signal=b)
        kf = int(out["k_found"][b])
        assert int(out["status"][b]) == ref.status and kf == ref.freqs.shape[0]
        assert np.array_equal(out["freqs"][b, :kf], ref.freqs)
        tr = out["trace"][b, :ref.rounds]
        want = np.array([[t["i"], t["kstar"], t["p"], t["m"], t["n_cand"], t["n_acc"],
                          t["n_R"], t["verify"]] for t in ref.trace])
        assert np.array_equal(tr, want)
    plan.close()


def _recover_stats(pb, plan):
    import torch
    sfft = _sfft()
    out = sfft.outputs_to_host(sfft.sfft_recover(plan, sfft.DeviceBatch.from_planted(pb)))
    torch.cuda.synchronize()
    ok = 0
    for b in range(pb.B):
        w, _ = pb.signal(b)
        kf = int(out["k_found"][b])
        o = np.lexsort(w.T[::-1])
        ok += int(out["status"][b] == 0 and kf == w.shape[0]
                  and np.array_equal(out["freqs"][b, :kf], w[o]))
    return ok / pb.B, float(np.mean(out["rounds"])), float(np.mean(out["samples"]))


def test_learned_classifier_gain():
    """What the trained network gains: on held-out noisy signals of the training
    distribution (sigma ~ U[0, 1e-2], tau = 1e-3), the learned test keeps exact
    support on every signal while needing far fewer rounds and samples than the
    plain ratio test, whose fixed tolerance rejects noisy singletons."""
    sfft = _sfft()
    from paper_1606_07407_amd import classifier as cls
    x, y, _ = cls.export_features(1_000_000)
    w, hist = cls.train(x, y)
    acc = cls.accuracy(w, x, y)
    _say(f"[gain] trained on {x.shape[0]} buckets: loss {hist[0]:.4f} -> {hist[-1]:.4f}, "
         f"accuracy {acc:.4f}")
    assert acc > 0.98
    del x, y
    cfg, pb = _c4_batch(64, 2000, seed_off=90000)
    plain = _plan(cfg, 2000, pb.B)
    learned = _plan(cfg, 2000, pb.B, classifier=sfft.SFFT_CLS_MLP, mlp_weights=w,
                    mlp_threshold=0.5)
    sp, rp, np_ = _recover_stats(pb, plain)
    sl, rl, nl = _recover_stats(pb, learned)
    _say(f"[gain] plain: success {sp:.3f}, rounds {rp:.2f}, samples {np_:.0f}; "
         f"learned: success {sl:.3f}, rounds {rl:.2f}, samples {nl:.0f}")
    assert sl == 1.0 and sl >= sp
    assert rl <= 0.6 * rp
    assert nl < np_
    plain.close()
    learned.close()
