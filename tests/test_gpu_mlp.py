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


def _abs_grad(oracle, params, x, base, target):
    """Per-parameter bounds of the gradient's terms, from the oracle's
    forward pass: G = the backward contraction over absolute values (sum
    over samples of |each sample's contribution|, so |g| <= G), and M = the
    largest single sample's such contribution."""
    y, cache = oracle.mlp_forward(params, x, base)
    n = y.size
    dz = np.abs(2.0 * (y - np.asarray(target, np.float64)) / n)[:, None]
    G, M = [], []
    for li in range(len(cache) - 1, -1, -1):
        ar, Wr, z = cache[li]
        if li < len(cache) - 1:
            dz = dz * (z > 0)
        per = dz[:, :, None] * np.abs(ar)[:, None, :]       # n x out x in
        G.append((per.sum(0).reshape(-1), dz.sum(0)))
        M.append((per.max(0).reshape(-1), dz.max(0)))
        dz = dz @ np.abs(Wr)
    flat = lambda L: np.concatenate([v for pair in reversed(L) for v in pair])
    return flat(G), flat(M)


def _grid_case(oracle, rng, n):
    """Inputs and parameters on power-of-two grids chosen so that every
    forward dot product is exact in fp32 whatever the summation order (the
    test checks it below): then the GPU's fp32 layers and the oracle's fp64
    layers see the same values before every bfloat16 rounding and every
    ReLU, and round them the same way."""
    dims = oracle.MLP_DIMS
    p = []
    for i in range(len(dims) - 1):
        n_in, n_out = dims[i], dims[i + 1]
        W = rng.integers(-2, 3, size=(n_out, n_in)) * 2.0 ** -5
        if i >= 2:
            W = W * (rng.random(W.shape) < 0.25)     # sparse deeper layers
        b = rng.integers(-4, 5, size=n_out) * 2.0 ** -6
        p += [W.reshape(-1), b]
    p = np.concatenate(p)
    x = rng.integers(-8, 9, size=(n, 20)) * 2.0 ** -2
    base = rng.integers(0, 64, size=n) * 2.0 ** -6
    t = base + rng.integers(-16, 17, size=n) * 2.0 ** -6
    # exactness of the forward sums: every term of a layer's dot products
    # is a multiple of a power of two q, and their absolute sum stays below
    # 2^24 q, so every partial sum is an exact fp32 value
    def grain(v):
        v = np.abs(np.asarray(v, np.float64).reshape(-1))
        v = v[v > 0]
        q = 1.0
        while v.size and np.any(np.mod(v, q) != 0):
            q /= 2
        return q

    _, cache = oracle.mlp_forward(p, x, base)
    for (W, b), (ar, Wr, z) in zip(oracle.mlp_unpack(p), cache):
        q = min(grain(ar) * grain(Wr), grain(b))
        bound = (np.abs(ar) @ np.abs(Wr).T + np.abs(b)).max()
        assert bound < 2.0 ** 24 * q, (bound, q)
    # the output y = base + z is exact in fp32 too
    z = cache[-1][2][:, 0]
    q = min(grain(base), grain(z))
    assert (np.abs(base) + np.abs(z)).max() < 2.0 ** 24 * q
    f32 = lambda a: np.asarray(a, np.float32)
    return f32(p), f32(x), f32(base), f32(t)


@gpu
@pytest.mark.parametrize("n", [1, 33, 300, 512])
def test_gradients_exact_grid(oracle, n):
    """Element-wise gradient parity.  On grid inputs (see _grid_case) the
    forward pass is the oracle's exactly (y compared for equality), so the
    only differences left are the fp32 roundings of the backward products
    and sums: each gradient element is a sum of at most n * 64 products
    along paths of at most ~700 roundings, so |g - g_ref| <= 2^-13 G with G
    the same contraction over absolute values (gamma_k = k u, u = 2^-24)."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(4000 + n)
    p0, x, base, t = _grid_case(oracle, rng, n)
    print("[case] mlp grid n", n, flush=True)
    m = C.MLP(p0)
    xd, bd, td = (torch.from_numpy(a).cuda() for a in (x, base, t))
    y = m.forward(xd, bd)
    loss = m.train_step(xd, bd, td, lr=0.0)
    torch.cuda.synchronize()
    pd = p0.astype(np.float64)
    y_ref, _ = oracle.mlp_forward(pd, x, base)
    assert np.array_equal(y.cpu().numpy().astype(np.float64), y_ref)
    l_ref, g_ref = oracle.mlp_loss_grad(pd, x, base, t)
    assert abs(loss.item() - l_ref) <= 2.0 ** -20 * max(1.0, l_ref)
    g = m.read(1).astype(np.float64)
    G, _ = _abs_grad(oracle, pd, x, base, t)
    bad = np.abs(g - g_ref) > 2.0 ** -13 * G + 1e-30
    assert not np.any(bad), (np.flatnonzero(bad)[:10], g[bad][:10], g_ref[bad][:10])
    m.close()


@gpu
@pytest.mark.parametrize("n", [1, 33, 300, 512])
def test_forward_and_gradients(oracle, n):
    """Random (off-grid) inputs.  Forward sums round in fp32 on the GPU,
    so a value next to a bfloat16 rounding boundary can round to the
    neighbouring bfloat16 on one side (a relative change of at most 2^-7 of
    that activation, for that sample).  Element-wise bound: the fp32 term
    2^-13 G, plus 2^-4 M for such changes (M = the largest single sample's
    absolute contribution to the element), plus 1e-3 |g_ref|."""
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
    G, M = _abs_grad(oracle, p0.astype(np.float64), x, base, t)
    tol = 2.0 ** -13 * G + 2.0 ** -4 * M + 1e-3 * np.abs(g_ref) + 1e-30
    bad = np.abs(g - g_ref) > tol
    assert not np.any(bad), (np.flatnonzero(bad)[:10], g[bad][:10], g_ref[bad][:10])
    # one Adam step from zero state
    m.train_step(xd, bd, td, lr=1e-3)
    torch.cuda.synchronize()
    g1 = m.read(1).astype(np.float64)
    p1 = m.read(0).astype(np.float64)
    p_ref, _, _ = oracle.adam_step(p0.astype(np.float64), 0 * g1, 0 * g1, g1, 1, lr=1e-3)
    assert np.allclose(p1, p_ref, rtol=1e-5, atol=1e-6)
    m.close()


@gpu
@pytest.mark.parametrize("d", [5, 7, 11])
def test_features_match_reference(oracle, d):
    """Features from the 128-bit rows at odd d (order-statistic positions
    round(k (d - 1) / 6)) against the oracle's."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    print("[case] features d", d, flush=True)
    q = W.job6a(seed=21, scale=0.003, d=d, w=512)
    dq = C.DeviceQuery(q)
    dq.build()
    masks = oracle.connected_subplans(5, q.edge_u, q.edge_v)
    row_est, est, flags = dq.estimate(masks)
    shape = oracle.shape_stats(5, q.edge_u, q.edge_v, masks)
    md = torch.tensor(np.asarray(masks, dtype=np.uint64).view(np.int64), device="cuda")
    x, base = C.features(row_est, est, md, dq.n_selected, 5, q.edge_u, q.edge_v)
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


@gpu
def test_feature_shapes_on_large_graphs(oracle):
    """The kernel's 5 shape features (tables, edges, diameter, largest
    degree, cycles) against the oracle's all-pairs shortest paths, on
    random connected sub-plans of a 17-table join graph with extra edges
    (cycles), and on a 6-cycle with chords."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(17)
    n = 17
    eu, ev = [], []
    for t in range(1, n):
        eu.append(int(rng.integers(0, t)))
        ev.append(t)
    for _ in range(6):
        a, b = rng.choice(n, size=2, replace=False)
        eu.append(int(a))
        ev.append(int(b))
    masks = W.connected_masks(n, eu, ev, max_tables=9)
    masks = [masks[i] for i in rng.choice(len(masks), size=min(3000, len(masks)),
                                          replace=False)]
    graphs = [(n, eu, ev, masks),
              (6, [0, 1, 2, 3, 4, 5, 0, 1, 2], [1, 2, 3, 4, 5, 0, 3, 4, 5],
               W.connected_masks(6, [0, 1, 2, 3, 4, 5, 0, 1, 2],
                                 [1, 2, 3, 4, 5, 0, 3, 4, 5]))]
    for (nt, gu, gv, ms) in graphs:
        print("[case] feature shapes", nt, len(gu), len(ms), flush=True)
        k = len(ms)
        d = 3
        row_est = torch.zeros((k, d, 2), dtype=torch.int64, device="cuda")
        est = torch.zeros(k, dtype=torch.float64, device="cuda")
        nsel = torch.ones(nt, dtype=torch.int64, device="cuda")
        md = torch.tensor(np.asarray(ms, dtype=np.uint64).view(np.int64), device="cuda")
        x, base = C.features(row_est, est, md, nsel, nt, gu, gv)
        torch.cuda.synchronize()
        ref = oracle.shape_stats(nt, gu, gv, ms)
        assert np.array_equal(x[:, 15:].cpu().numpy().astype(np.float64), ref)


@gpu
def test_checkpoint_resumes_training_exactly(oracle, tmp_path):
    """A checkpoint (parameters, Adam moments, step count) written after some
    steps and loaded into a new network: both continue identically, bit
    for bit, through further Adam steps."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(8)
    x, base, t = _data(rng, 1024)
    xd, bd, td = (torch.from_numpy(a).cuda() for a in (x, base, t))
    m1 = C.MLP(oracle.mlp_init(2).astype(np.float32))
    print("[case] mlp checkpoint", flush=True)
    for k in range(5):
        m1.train_step(xd[k * 200:(k + 1) * 200].contiguous(),
                      bd[k * 200:(k + 1) * 200].contiguous(),
                      td[k * 200:(k + 1) * 200].contiguous(), 1e-3)
    path = str(tmp_path / "ckpt.npz")
    m1.save(path)
    m2 = C.MLP.load(path)
    assert m2.adam_steps() == m1.adam_steps() == 5
    for k in range(3):
        for m in (m1, m2):
            m.train_step(xd[:300].contiguous(), bd[:300].contiguous(),
                         td[:300].contiguous(), 1e-3)
    torch.cuda.synchronize()
    for what in (0, 2, 3):
        assert np.array_equal(m1.read(what), m2.read(what)), what
    m1.close()
    m2.close()
