"""Weighted min-sum BP+DC (learned per-edge scales): forward parity with the
float32 oracle, reduction to plain scaled min-sum, and the adjoint kernel
against central finite differences of the float64 oracle (GPU)."""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import oracle_params

pytestmark = pytest.mark.gpu

T = (25, 25)


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_08695_amd as P
    code = synth.bb_code("bb144", p=0.05)
    prm = P.Params(max_iter=T, alpha=0.625, stop_on_converge=False, seed=21)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_GROUP)
    return P, code, prm, plan


def _run_fwd(plan, code, syndromes, w, ckpt_every=5):
    import torch
    syn = torch.from_numpy(synth.pack_bits(syndromes).view(np.int64)).cuda()
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    out = plan.wms_forward(wt, syn, ckpt_every=ckpt_every)
    torch.cuda.synchronize()
    return syn, wt, out


@pytest.mark.parametrize("kind", ["uniform", "random"])
def test_weighted_forward_bit_exact_vs_float32_oracle(setup, kind):
    P, code, prm, plan = setup
    shots = synth.make_shots(code, 300, 5001)
    E = code.H.nnz
    rng = np.random.default_rng(1)
    w = np.full(2 * E, 0.625) if kind == "uniform" else 0.625 + 0.1 * rng.standard_normal(2 * E)
    w = w.astype(np.float32)
    syn, wt, out = _run_fwd(plan, code, shots.syndromes, w)
    ref = oracle.decode(code, shots.syndromes, oracle_params(prm, "channel"), precision="f32",
                        weights=w.astype(np.float64), want_post1=True)
    post = out["post"].cpu().numpy()
    flags = out["flags"].cpu().numpy()
    cut = synth.unpack_bits(out["cut"].cpu().numpy().view(np.uint64), code.n)
    np.testing.assert_array_equal(flags, ref["flags"])
    np.testing.assert_array_equal(cut, ref["cut"])
    np.testing.assert_array_equal(post[0].view(np.uint32), ref["post1"].astype(np.float32).view(np.uint32))
    dc = (ref["flags"] & 2) != 0
    assert dc.sum() > 5
    np.testing.assert_array_equal(post[1][dc].view(np.uint32),
                                  ref["post"][dc].astype(np.float32).view(np.uint32))
    if kind == "uniform":
        # weights all equal to the scale reproduce the unweighted decoder (fixed iterations)
        plan2 = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_LANE)
        from gpu_helpers import gpu_decode
        g = gpu_decode(plan2, code, shots.syndromes)
        np.testing.assert_array_equal(g["flags"], flags)
        np.testing.assert_array_equal(g["cut"], cut)


def _loss_and_grad_post(post, errors, cut, flags):
    """Mean over shots of BCE(pass-1 posteriors, e) + [DC] * BCE(pass-2 posteriors on
    non-cut columns, e), BCE in LLR form e*softplus(L) + (1-e)*softplus(-L)."""
    e = errors.astype(np.float64)
    B, n = e.shape
    L1, L2 = post[0].astype(np.float64), post[1].astype(np.float64)
    dc = ((flags & 2) != 0)[:, None]
    keep2 = dc & (cut == 0)
    L2 = np.where(keep2, L2, 0.0)

    def bce(L):
        return e * np.logaddexp(0, L) + (1 - e) * np.logaddexp(0, -L)

    def dbce(L):
        return 1.0 / (1.0 + np.exp(-L)) - (1 - e)

    loss = (bce(L1).sum() + (bce(L2) * keep2).sum()) / B
    g = np.stack([dbce(L1) / B, np.where(keep2, dbce(L2), 0.0) / B])
    return loss, g


# checkpoints every iteration (the adjoint reads each back) and every 5 (segments recomputed)
@pytest.mark.parametrize("ckpt_every", [1, 5])
def test_adjoint_matches_finite_differences_of_float64_oracle(setup, ckpt_every):
    import torch
    P, code, prm, plan = setup
    B = 256
    shots = synth.make_shots(code, B, 5002)
    E = code.H.nnz
    rng = np.random.default_rng(2)
    w = (0.625 + 0.05 * rng.standard_normal(2 * E)).astype(np.float32)
    syn, wt, out = _run_fwd(plan, code, shots.syndromes, w, ckpt_every)
    post = out["post"].cpu().numpy()
    flags = out["flags"].cpu().numpy()
    cut = synth.unpack_bits(out["cut"].cpu().numpy().view(np.uint64), code.n)
    _, gpost = _loss_and_grad_post(post, shots.errors, cut, flags)
    gw = plan.wms_backward(wt, syn, out, torch.from_numpy(gpost.astype(np.float32)).cuda()).cpu().numpy()
    op = oracle_params(prm, "channel")

    def f64_loss(wv):
        o = oracle.decode(code, shots.syndromes, op, precision="f64", weights=wv, want_post1=True)
        post64 = np.stack([o["post1"], o["post"]])
        return _loss_and_grad_post(post64, shots.errors, o["cut"], o["flags"])[0], o["cut"]

    w64 = w.astype(np.float64)
    base, base_cut = f64_loss(w64)
    idx = rng.choice(2 * E, size=48, replace=False)
    checked = 0
    for j in idx:
        h = 1e-4 * max(1.0, abs(w64[j]))
        wp, wm = w64.copy(), w64.copy()
        wp[j] += h
        wm[j] -= h
        lp, cp = f64_loss(wp)
        lm, cm = f64_loss(wm)
        if not ((cp == base_cut).all() and (cm == base_cut).all()):
            continue  # the cut changed: a kink of the piecewise-smooth loss
        fwd, bwd = (lp - base) / h, (base - lm) / h
        if abs(fwd - bwd) > 1e-3 * max(1e-3, abs(fwd) + abs(bwd)):
            continue  # a min / sign switch inside [w - h, w + h]
        fd = (lp - lm) / (2 * h)
        assert abs(gw[j] - fd) <= 2e-3 * max(abs(fd), 1e-3), (j, gw[j], fd)
        checked += 1
    assert checked >= 24, checked
    assert np.isfinite(gw).all() and np.abs(gw).max() > 0


def test_autograd_function_and_training_step_reduce_loss(setup):
    import torch
    P, code, prm, plan = setup
    f = P.weighted_bpdc(plan, ckpt_every=5)
    E = code.H.nnz
    w = torch.full((2 * E,), 0.625, dtype=torch.float32, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-2)
    losses = []
    for step in range(12):
        sh = synth.make_shots(code, 512, 7000 + step % 3)
        syn = torch.from_numpy(synth.pack_bits(sh.syndromes).view(np.int64)).cuda()
        e = torch.from_numpy(sh.errors.astype(np.float32)).cuda()
        post, cut, flags = f(w, syn)
        dc = ((flags & 2) != 0).float()[:, None]
        cutb = torch.from_numpy(synth.unpack_bits(cut.cpu().numpy().view(np.uint64), code.n)).cuda()
        keep2 = dc * (1 - cutb.float())
        L1 = post[0]
        L2 = torch.where(keep2 > 0, post[1], torch.zeros_like(post[1]))
        bce = lambda L: e * torch.nn.functional.softplus(L) + (1 - e) * torch.nn.functional.softplus(-L)
        loss = (bce(L1).sum() + (bce(L2) * keep2).sum()) / e.shape[0]
        opt.zero_grad()
        loss.backward()
        assert w.grad is not None and torch.isfinite(w.grad).all()
        opt.step()
        losses.append(loss.item())
    assert np.mean(losses[-3:]) < np.mean(losses[:3])


def _loss_final(post2, errors, cut):
    """Mean over shots of BCE(final posteriors, e) on the uncut columns, every shot included:
    a shot without DC reports its first-pass posteriors in the final row, so this loss
    reaches the first pass's scales through those shots."""
    e = errors.astype(np.float64)
    keep = cut == 0
    L = np.where(keep, post2.astype(np.float64), 0.0)
    bce = e * np.logaddexp(0, L) + (1 - e) * np.logaddexp(0, -L)
    g = np.where(keep, 1.0 / (1.0 + np.exp(-L)) - (1 - e), 0.0) / e.shape[0]
    return float((bce * keep).sum() / e.shape[0]), g


def test_adjoint_of_a_loss_on_the_final_row_of_every_shot(setup):
    import torch
    P, code, prm, plan = setup
    B = 192
    shots = synth.make_shots(code, B, 5003)
    E = code.H.nnz
    rng = np.random.default_rng(3)
    w = (0.625 + 0.05 * rng.standard_normal(2 * E)).astype(np.float32)
    syn, wt, out = _run_fwd(plan, code, shots.syndromes, w)
    post = out["post"].cpu().numpy()
    flags = out["flags"].cpu().numpy()
    cut = synth.unpack_bits(out["cut"].cpu().numpy().view(np.uint64), code.n)
    assert ((flags & 2) == 0).sum() > B // 2 and ((flags & 2) != 0).sum() > 5
    _, g2 = _loss_final(post[1], shots.errors, cut)
    gpost = np.stack([np.zeros_like(g2), g2]).astype(np.float32)
    gw = plan.wms_backward(wt, syn, out, torch.from_numpy(gpost).cuda()).cpu().numpy()
    op = oracle_params(prm, "channel")

    def f64_loss(wv):
        o = oracle.decode(code, shots.syndromes, op, precision="f64", weights=wv)
        return _loss_final(o["post"], shots.errors, o["cut"])[0], o["cut"]

    w64 = w.astype(np.float64)
    base, base_cut = f64_loss(w64)
    # first-pass scales (reached through the shots without DC) and second-pass scales
    idx = np.concatenate([rng.choice(E, size=24, replace=False), E + rng.choice(E, size=12, replace=False)])
    checked = [0, 0]
    for j in idx:
        h = 1e-4 * max(1.0, abs(w64[j]))
        wp, wm = w64.copy(), w64.copy()
        wp[j] += h
        wm[j] -= h
        lp, cp = f64_loss(wp)
        lm, cm = f64_loss(wm)
        if not ((cp == base_cut).all() and (cm == base_cut).all()):
            continue
        fwd, bwd = (lp - base) / h, (base - lm) / h
        if abs(fwd - bwd) > 1e-3 * max(1e-3, abs(fwd) + abs(bwd)):
            continue
        fd = (lp - lm) / (2 * h)
        assert abs(gw[j] - fd) <= 2e-3 * max(abs(fd), 1e-3), (j, gw[j], fd)
        checked[int(j >= E)] += 1
    assert checked[0] >= 12 and checked[1] >= 4, checked
    assert np.abs(gw[:E]).max() > 0


def _balanced_code(m, R, dv, d_rows, d_weight, p, seed):
    """Every column meets dv distinct checks of lowest current degree (rows of exactly R edges);
    D: d_rows random column subsets of weight d_weight."""
    n = m * R // dv
    rng = np.random.default_rng(seed)
    deg = np.zeros(m, dtype=np.int64)
    H = np.zeros((m, n), dtype=np.uint8)
    for v in rng.permutation(n):
        for c in np.argsort(deg * m + rng.permutation(m))[:dv]:
            H[c, v] = 1
            deg[c] += 1
    D = np.zeros((d_rows, n), dtype=np.uint8)
    for i in range(d_rows):
        D[i, rng.choice(n, size=d_weight, replace=False)] = 1
    return synth.Code(f"balanced_m{m}_r{R}_dv{dv}", synth.Csr.from_dense(H), synth.Csr.from_dense(D),
                      np.full(n, p), None, "channel")


# the weighted kernels are compiled for three degree classes (columns / rows of at most 3 / 6, the
# BB codes above; 4 / 8; 16 / 21): an HGP code (rows of 7, columns of 3 and 4) and a synthetic code
# with rows of 12 and columns of 5 run the other two.  Per code: (builder, iterations per pass,
# finite-difference step).  Rows of 12 make the loss far less smooth at 15 iterations (most
# coordinates then have a min switch within any usable step), so that code runs 6 + 6 with a
# smaller step.
DEGREE_CODES = {
    "hgp_rows7": (lambda: synth.hgp_code(synth.random_regular_classical(12, 4400), name="hgp_w", p=0.05,
                                         with_logicals=False), 15, 1e-4),
    "rows12_cols5": (lambda: _balanced_code(60, 12, 5, 60, 6, 0.03, 4401), 6, 1e-5),
}


@pytest.mark.parametrize("name", list(DEGREE_CODES))
def test_weighted_degree_classes(name):
    import torch
    import paper_2510_08695_amd as P
    build, iters, step = DEGREE_CODES[name]
    code = build()
    prm = P.Params(max_iter=(iters, iters), alpha=0.625, stop_on_converge=False, seed=23)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_GROUP)
    E = code.H.nnz
    print(f"case weighted {name}: rows <= {code.H.row_weights().max()}, columns <= {code.H.col_weights().max()}",
          flush=True)
    rng = np.random.default_rng(5)
    # forward: bit-exact with the float32 oracle on the same per-edge scales
    shots = synth.make_shots(code, 200, 5101)
    w = (0.625 + 0.1 * rng.standard_normal(2 * E)).astype(np.float32)
    syn, wt, out = _run_fwd(plan, code, shots.syndromes, w, 1)
    ref = oracle.decode(code, shots.syndromes, oracle_params(prm, "channel"), precision="f32",
                        weights=w.astype(np.float64), want_post1=True)
    post = out["post"].cpu().numpy()
    flags = out["flags"].cpu().numpy()
    cut = synth.unpack_bits(out["cut"].cpu().numpy().view(np.uint64), code.n)
    np.testing.assert_array_equal(flags, ref["flags"])
    np.testing.assert_array_equal(cut, ref["cut"])
    np.testing.assert_array_equal(post[0].view(np.uint32), ref["post1"].astype(np.float32).view(np.uint32))
    dc = (ref["flags"] & 2) != 0
    assert dc.sum() > 3
    np.testing.assert_array_equal(post[1][dc].view(np.uint32), ref["post"][dc].astype(np.float32).view(np.uint32))
    # adjoint: central finite differences of the float64 oracle's loss (checkpoints every iteration)
    _, gpost = _loss_and_grad_post(post, shots.errors, cut, flags)
    gw = plan.wms_backward(wt, syn, out, torch.from_numpy(gpost.astype(np.float32)).cuda()).cpu().numpy()
    op = oracle_params(prm, "channel")

    def f64_loss(wv):
        o = oracle.decode(code, shots.syndromes, op, precision="f64", weights=wv, want_post1=True)
        return _loss_and_grad_post(np.stack([o["post1"], o["post"]]), shots.errors, o["cut"], o["flags"])[0], o["cut"]

    w64 = w.astype(np.float64)
    base, base_cut = f64_loss(w64)
    checked = 0
    for j in rng.choice(2 * E, size=32, replace=False):
        h = step * max(1.0, abs(w64[j]))
        wp, wm = w64.copy(), w64.copy()
        wp[j] += h
        wm[j] -= h
        lp, cp = f64_loss(wp)
        lm, cm = f64_loss(wm)
        if not ((cp == base_cut).all() and (cm == base_cut).all()):
            continue
        fwd, bwd = (lp - base) / h, (base - lm) / h
        if abs(fwd - bwd) > 1e-3 * max(1e-3, abs(fwd) + abs(bwd)):
            continue
        fd = (lp - lm) / (2 * h)
        assert abs(gw[j] - fd) <= 2e-3 * max(abs(fd), 1e-3), (j, gw[j], fd)
        checked += 1
    assert checked >= 16, checked
