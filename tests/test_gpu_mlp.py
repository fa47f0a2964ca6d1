"""Learned correction kernels against the FP64 oracle: forward values,
gradients (BF16 tolerance), one Adam step, features from 128-bit rows."""
import numpy as np
import pytest

from paper_2102_02440_amd import workloads as W

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _data(rng, n):
    x = rng.normal(size=(n, 20)).astype(np.float32) * 3
    base = rng.uniform(0, 20, size=n).astype(np.float32)
    t = (base + rng.normal(size=n)).astype(np.float32)
    return x, base, t


@gpu
@pytest.mark.parametrize("n", [1, 33, 300, 512])
def test_forward_and_gradients(oracle, n):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(n)
    p0 = oracle.mlp_init(7)
    p0[-65:] = rng.normal(size=65) * 0.2      # non-zero output layer
    p0 = p0.astype(np.float32)
    x, base, t = _data(rng, n)
    print("[case] mlp n", n, flush=True)
    m = C.MLP(p0)
    xd, bd, td = (torch.from_numpy(a).cuda() for a in (x, base, t))
    y = m.forward(xd, bd)
    loss = m.train_step(xd, bd, td, lr=0.0)
    torch.cuda.synchronize()
    y_ref, _ = oracle.mlp_forward(p0.astype(np.float64), x, base)
    assert np.allclose(y.cpu().numpy(), y_ref, rtol=1e-3, atol=2e-2)
    l_ref, g_ref = oracle.mlp_loss_grad(p0.astype(np.float64), x, base, t)
    assert abs(loss.item() - l_ref) <= 2e-2 * max(1.0, l_ref)
    g = m.read(1).astype(np.float64)
    err = np.linalg.norm(g - g_ref) / max(1e-12, np.linalg.norm(g_ref))
    assert err < 2e-2, err
    # one Adam step from zero state
    m.train_step(xd, bd, td, lr=1e-3)
    torch.cuda.synchronize()
    g1 = m.read(1).astype(np.float64)
    p1 = m.read(0).astype(np.float64)
    p_ref, _, _ = oracle.adam_step(p0.astype(np.float64), 0 * g1, 0 * g1, g1, 1, lr=1e-3)
    assert np.allclose(p1, p_ref, rtol=1e-5, atol=1e-6)
    m.close()


@gpu
def test_features_match_reference(oracle):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    q = W.job6a(seed=21, scale=0.003, d=7, w=512)
    dq = C.DeviceQuery(q)
    dq.build()
    masks = oracle.connected_subplans(5, q.edge_u, q.edge_v)
    row_est, est, flags = dq.estimate(masks)
    shape = C.shape_stats(5, q.edge_u, q.edge_v, masks)
    md = torch.tensor(np.asarray(masks, dtype=np.uint64).view(np.int64), device="cuda")
    x, base = C.features(row_est, est, md, dq.n_selected, 5, torch.from_numpy(shape).cuda())
    torch.cuda.synchronize()
    rows = C.row_values(row_est)
    n_sel = dq.n_selected.cpu().tolist()
    for k, mk in enumerate(masks):
        signed = [r - (1 << 128) if r >> 127 else r for r in rows[k]]
        xr, br = oracle.mlp_features(signed, est.cpu().numpy()[k],
                                     [n_sel[t] for t in range(5) if mk >> t & 1], shape[k])
        assert np.allclose(x[k].cpu().numpy(), xr, rtol=1e-6, atol=1e-6), k
        assert abs(base[k].item() - br) <= 1e-6 * max(1, br)


@gpu
def test_training_fits_a_correction():
    """Training with the HIP kernels learns a correction that the raw base
    misses: loss falls well below its starting value."""
    torch = _torch()
    from oracle import oracle as o
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(3)
    n = 4096
    x = rng.normal(size=(n, 20)).astype(np.float32)
    base = rng.uniform(0, 10, size=n).astype(np.float32)
    t = (base + 1.5 * np.tanh(x[:, 0]) - 0.7 * x[:, 3] * (x[:, 4] > 0)).astype(np.float32)
    m = C.MLP(o.mlp_init(5).astype(np.float32))
    xd, bd, td = (torch.from_numpy(a).cuda() for a in (x, base, t))
    first = None
    for ep in range(40):
        perm = torch.randperm(n, device="cuda")
        for s in range(0, n, 512):
            idx = perm[s:s + 512]
            loss = m.train_step(xd[idx].contiguous(), bd[idx].contiguous(),
                                td[idx].contiguous(), lr=3e-3)
            if first is None:
                first = loss.item()
    m.train_step(xd, bd, td, lr=0.0)
    final = m._loss.item()
    print("[case] training loss", first, "->", final, flush=True)
    assert final < 0.2 * first


@gpu
def test_train_epoch_matches_steps(oracle):
    """One epoch through compass_mlp_train_epoch (rows gathered through a
    permutation inside the kernels) equals the same batches trained one
    compass_mlp_train_step at a time on gathered copies: parameters, Adam
    state and per-batch losses bit for bit; a ragged tail is left out."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(5)
    n, batch = 2000, 300
    x, base, t = _data(rng, n)
    p0 = oracle.mlp_init(3).astype(np.float32)
    xd, bd, td = (torch.from_numpy(a).cuda() for a in (x, base, t))
    perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).cuda()
    print("[case] mlp epoch", n, batch, flush=True)
    m1 = C.MLP(p0)
    losses = m1.train_epoch(xd, bd, td, perm, batch, 1e-3)
    m2 = C.MLP(p0)
    ref = []
    for k in range(n // batch):
        idx = perm[k * batch:(k + 1) * batch].long()
        ref.append(m2.train_step(xd[idx].contiguous(), bd[idx].contiguous(),
                                 td[idx].contiguous(), 1e-3).item())
    torch.cuda.synchronize()
    assert losses.numel() == n // batch
    assert np.array_equal(losses.cpu().numpy(), np.asarray(ref, dtype=np.float32))
    for what in (0, 2, 3):
        assert np.array_equal(m1.read(what), m2.read(what)), what
    m1.close()
    m2.close()
