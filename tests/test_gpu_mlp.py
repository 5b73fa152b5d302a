"""Warm-start network kernels vs the FP64 CPU oracle, through the C ABI (run on
an MI355X).

Tolerances.  The kernels read bfloat16 weights and sum in FP32; the oracle
uses the same bfloat16 values in FP64.  Dot products of at most 256 terms in
FP32 carry a relative error of a few 1e-7 of the sum of absolute terms, so
outputs are compared at 2e-5 of the largest output magnitude and gradients at
2e-4 of each tensor's largest entry.  The max over points is an argmax: inputs
are chosen (by seed) so that every channel's top two pre-activations differ by
more than 1e-3 in the oracle, so both sides route each gradient to the same
point.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp_oracle as M  # noqa: E402
from paper_2606_10019_amd import gcvo, synth, warmstart  # noqa: E402

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def weights(seed):
    w32 = warmstart.Network.init_weights(seed)
    rng = np.random.default_rng(seed + 100)
    w32 = w32 + (rng.normal(size=w32.shape) * 0.05).astype(np.float32)     # non-zero biases too
    return M.bf16_round(w32.astype(np.float32)).astype(np.float64), w32


def problem(seed, B=5, P=300, min_size=100):
    """Ragged clouds (smaller than P when min_size < P: rows then repeat),
    subsample indices, source motions, labels; re-drawn until every channel's
    argmax is unambiguous in the oracle (exact ties between repeated rows are
    resolved identically on both sides: first position wins)."""
    for attempt in range(50):
        rng = np.random.default_rng(1000 * seed + attempt)
        sizes_t = rng.integers(min_size, 900, size=B)
        sizes_s = rng.integers(min_size, 900, size=B)
        tgt = [rng.normal(size=(n, 3)).astype(np.float32) * 5 for n in sizes_t]
        src = [rng.normal(size=(n, 3)).astype(np.float32) * 5 for n in sizes_s]
        tidx = np.stack([rng.choice(n, P, replace=n < P) for n in sizes_t]).astype(np.int32)
        sidx = np.stack([rng.choice(n, P, replace=n < P) for n in sizes_s]).astype(np.int32)
        mot = np.stack([warmstart.planar_motion(rng)[:3, :].reshape(-1) for _ in range(B)]).astype(np.float32)
        tmot = np.stack([warmstart.planar_motion(rng)[:3, :].reshape(-1) for _ in range(B)]).astype(np.float32)
        Y = rng.normal(size=(B, 6)).astype(np.float32)
        w64, w32 = weights(seed)
        S, T = M.gather_inputs(src, tgt, sidx, tidx, mot.astype(np.float64), 4.0, tmot.astype(np.float64))
        p = M.unpack(w64)
        ok = True
        for pts in S + T:
            _, _, _, h1, pre2 = M.cloud_feature(pts, p)
            top = np.sort(pre2, axis=0)[-2:]
            if np.any((top[1] - top[0] < 1e-3) & (top[1] - top[0] > 0) & (top[1] > 0)):
                ok = False
                break
        if ok:
            return dict(tgt=tgt, src=src, tidx=tidx, sidx=sidx, mot=mot, tmot=tmot, Y=Y, w64=w64, w32=w32, S=S, T=T)
    raise RuntimeError("no unambiguous draw")


def gpu_batch(pb, P=None):
    d = dev()
    tcat = torch.from_numpy(np.concatenate(pb["tgt"])).to(d)
    scat = torch.from_numpy(np.concatenate(pb["src"])).to(d)
    nt = np.array([len(a) for a in pb["tgt"]])
    ns = np.array([len(a) for a in pb["src"]])
    ts = np.concatenate([[0], np.cumsum(nt)[:-1]])
    ss = np.concatenate([[0], np.cumsum(ns)[:-1]])
    return gcvo.MlpBatch(tcat, ts, nt, scat, ss, ns, torch.from_numpy(pb["tidx"]).to(d),
                         torch.from_numpy(pb["sidx"]).to(d), torch.from_numpy(pb["tmot"]).to(d),
                         torch.from_numpy(pb["mot"]).to(d), 4.0)


def bf16_tensor(w64):
    return torch.from_numpy(warmstart.bf16_bits(w64.astype(np.float32)).view(np.int16)).to(dev())


def test_forward_and_poses_match_oracle():
    pb = problem(1)
    note("mlp forward 5 ragged pairs, P=300")
    out, T = gcvo.gcvo_mlp_forward(gpu_batch(pb), bf16_tensor(pb["w64"]), poses=True)
    assert T.is_cuda                      # predicted poses stay on the device
    T = T.cpu().numpy()
    ref = M.forward(pb["w64"], pb["S"], pb["T"])
    err = np.max(np.abs(out.cpu().numpy() - ref))
    note(f"  max |out - oracle| {err:.2e} (scale {np.max(np.abs(ref)):.2f})")
    assert err <= 2e-5 * max(1.0, np.max(np.abs(ref)))
    o = out.cpu().numpy().astype(np.float64)
    for b in range(len(o)):
        xi = np.concatenate([o[b, :3] * gcvo.GCVO_MLP_ROT_SCALE, o[b, 3:] * gcvo.GCVO_MLP_TRANS_SCALE])
        np.testing.assert_allclose(T[b], M.twist_to_pose(xi), atol=1e-12)


def test_loss_and_gradient_match_oracle():
    pb = problem(2, min_size=300)
    note("mlp loss/grad 5 ragged pairs, P=300")
    y = torch.from_numpy(pb["Y"]).to(dev())
    loss, grad = gcvo.gcvo_mlp_loss_grad(gpu_batch(pb), bf16_tensor(pb["w64"]), y)
    L, G = M.loss_and_grad(pb["w64"], pb["S"], pb["T"], pb["Y"].astype(np.float64))
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - L) <= 2e-5 * L
    gu, Gu = M.unpack(g), M.unpack(G)
    for name, _ in M.SHAPES:
        scale = np.max(np.abs(Gu[name]))
        err = np.max(np.abs(gu[name] - Gu[name]))
        note(f"  {name}: max err {err:.2e} of {scale:.2e}")
        assert err <= 2e-4 * scale + 1e-12, name
    # repeatable bit for bit
    _, grad2 = gcvo.gcvo_mlp_loss_grad(gpu_batch(pb), bf16_tensor(pb["w64"]), y)
    assert torch.equal(grad, grad2)


def test_adam_matches_oracle_and_rounds_to_bf16():
    rng = np.random.default_rng(5)
    n = gcvo.GCVO_MLP_N_PARAMS
    w0 = rng.normal(size=n).astype(np.float32)
    grads = [rng.normal(size=n).astype(np.float32) * s for s in (1.0, 0.1, 3.0)]
    d = dev()
    w = torch.from_numpy(w0.copy()).to(d)
    wb = torch.zeros(n, dtype=torch.int16, device=d)
    m, v = torch.zeros_like(w), torch.zeros_like(w)
    wr, mr, vr = w0.astype(np.float64), np.zeros(n), np.zeros(n)
    note("mlp adam 3 steps")
    for k, g in enumerate(grads, start=1):
        gcvo.gcvo_mlp_adam(w, wb, m, v, torch.from_numpy(g).to(d), k, 1e-2)
        wr, mr, vr = M.adam_step(wr, mr, vr, g.astype(np.float64), k, 1e-2)
    wg = w.cpu().numpy()
    assert np.max(np.abs(wg - wr)) <= 1e-6 * (1 + np.max(np.abs(wr)))
    bits = wb.cpu().numpy().view(np.uint16)
    assert np.array_equal(bits.astype(np.uint32) << 16, M.bf16_round(wg).view(np.uint32))


def test_index_out_of_range_is_rejected():
    pb = problem(3, B=2, P=64)
    pb["tidx"][1, 7] = len(pb["tgt"][1])            # one past the end of that cloud
    note("mlp forward with an out-of-range index")
    with pytest.raises(gcvo.GcvoError) as e:
        gcvo.gcvo_mlp_forward(gpu_batch(pb), bf16_tensor(pb["w64"]))
    assert e.value.status == gcvo.GCVO_ERR_INVALID


def test_training_reduces_loss():
    """A few hundred Adam steps on planes-and-cap pairs re-posed by random
    motions (labels exact by construction) cut the loss."""
    specs = [synth.make_config1(i, n=1500) for i in range(8)]
    ps = warmstart.PairSet.from_specs(specs, dev())
    labels = np.array([s.T_true for s in specs])
    net = warmstart.Network(warmstart.Network.init_weights(0), dev())
    note("mlp training 600 steps, batch 32")
    losses = warmstart.train(net, ps, labels, steps=600, batch=32, lr=1e-3, lr_final=5e-4, log_every=200,
                             log=note)
    first, last = np.mean(losses[:50]), np.mean(losses[-50:])
    note(f"  loss {first:.3f} -> {last:.3f}")
    assert last < 0.75 * first
