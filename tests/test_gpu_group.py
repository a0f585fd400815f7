"""Parity of the group kernel (one workgroup per shot, state in LDS), the
multi-code launch and its HIP-graph replay with the float32 oracle (GPU)."""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import assert_bit_exact, gpu_decode, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2510_08695_amd as P
    P.lib()
    return P


def _small_hgp(j, nc, p=0.05):
    return synth.hgp_code(synth.random_regular_classical(nc, 4100 + j), name=f"hgp{j}", p=p,
                          with_logicals=False)


CODES = {
    "toric6": lambda: synth.toric_code(6, p=0.07),
    "bb144": lambda: synth.bb_code("bb144", p=0.06),
    "hgp16": lambda: _small_hgp(0, 16, p=0.06),
    "phen_bb72_paper": lambda: synth.phenomenological_dem(synth.bb_code("bb72"), 4, 0.02, 0.02, True),
    "phen_bb72_open": lambda: synth.phenomenological_dem(synth.bb_code("bb72"), 4, 0.02, 0.02, False),
}


@pytest.mark.parametrize("name", list(CODES))
def test_group_kernel_bit_exact(P, name):
    code = CODES[name]()
    shots = synth.make_shots(code, 400, 31)
    sp = P.PRIOR_POSTERIOR if code.second_pass == "posterior" else P.PRIOR_CHANNEL
    prm = P.Params(max_iter=(40, 40), alpha=0.625, second_pass_prior=sp, seed=9)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_GROUP)
    print(f"case group {name} n={code.n} tile={plan.info(0)}", flush=True)
    g = gpu_decode(plan, code, shots.syndromes, shot_offset=11)
    ref = oracle.decode(code, shots.syndromes, oracle_params(prm, code.second_pass), precision="f32",
                        shot_offset=11)
    assert ((ref["flags"] & 2) != 0).sum() > 0
    assert_bit_exact(g, ref, code.n)


# one-wave workgroups on a code of more than 32 checks and 32 columns per thread (phenomenological
# BB144, T = 30: 2160 x 6480): the stop test reads the syndrome bits from LDS instead of a register
# and the second pass under the channel prior takes the variable phase that tests each column's cut
# bit; 1024 threads take the register paths on the same shots; both bit-exact with the oracle
@pytest.mark.parametrize("threads", [64, 1024])
def test_group_kernel_one_wave_workgroups_on_a_large_code(P, monkeypatch, threads):
    code = synth.phenomenological_dem(synth.bb_code("bb144"), 30, 0.01, 0.01, False)
    assert code.H.rows > 32 * 64 and code.n > 32 * 64 and code.H.rows <= 32 * 1024
    monkeypatch.setenv("BPDC_GROUP_THREADS", str(threads))
    shots = synth.make_shots(code, 200, 77)
    prm = P.Params(max_iter=(30, 30), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=9)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_GROUP)
    print(f"case group {threads} threads n={code.n} m={code.H.rows} tile={plan.info(0)}", flush=True)
    assert plan.info(0)["threads"] == threads
    g = gpu_decode(plan, code, shots.syndromes, shot_offset=3)
    ref = oracle.decode(code, shots.syndromes, oracle_params(prm, code.second_pass), precision="f32",
                        shot_offset=3)
    assert ((ref["flags"] & 2) != 0).sum() > 0
    assert_bit_exact(g, ref, code.n)


# single-code launches of small codes claim several consecutive shots at a time (toric L = 6,
# 72 columns: 8): one shot, batches that end inside the first claim or just past it, and a batch
# whose last claim straddles its end, all bit-exact at a nonzero shot offset
@pytest.mark.parametrize("B", [1, 7, 8, 9, 1001])
def test_group_kernel_claims_of_consecutive_shots(P, B):
    code = synth.toric_code(6, p=0.07)
    shots = synth.make_shots(code, B, 900 + B)
    prm = P.Params(max_iter=(30, 30), alpha=0.625, second_pass_prior=P.PRIOR_POSTERIOR, seed=9)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_GROUP)
    print(f"case group claims toric6 B={B}", flush=True)
    g = gpu_decode(plan, code, shots.syndromes, shot_offset=1_000_003)
    ref = oracle.decode(code, shots.syndromes, oracle_params(prm, "posterior"), precision="f32",
                        shot_offset=1_000_003)
    assert_bit_exact(g, ref, code.n)


def test_auto_plan_picks_lane_for_small_and_group_for_large(P):
    prm = P.Params(max_iter=(20, 20))
    small = P.Code.from_problem(synth.bb_code("bb144"))
    big = P.Code.from_problem(_small_hgp(1, 20))
    plan = P.Plan([small, big], prm, kernel=P.KERNEL_AUTO)
    assert plan.info(0)["kernel"] == P.KERNEL_LANE
    assert plan.info(1)["kernel"] == P.KERNEL_GROUP


def _mixed_batch(P, codes, counts, seed):
    import torch
    rng = np.random.default_rng(seed)
    code_of_shot = np.concatenate([np.full(k, i, np.int32) for i, k in enumerate(counts)])
    rng.shuffle(code_of_shot)
    syn_rows = [None] * len(code_of_shot)
    per_code = {}
    for i, c in enumerate(codes):
        idx = np.nonzero(code_of_shot == i)[0]
        sh = synth.make_shots(c, len(idx), seed + 1 + i)
        per_code[i] = (idx, sh)
        for k, b in enumerate(idx):
            syn_rows[b] = synth.pack_bits(sh.syndromes[k:k + 1])[0]
    syn = np.concatenate(syn_rows).view(np.int64)
    return code_of_shot, syn, per_code


def _run_multi(P, plan, codes, code_of_shot, syn, graph=False, replays=1):
    import torch
    cos = torch.from_numpy(code_of_shot).cuda()
    so, co, sw, nw = plan.multi_buffers(cos)
    syn_t = torch.from_numpy(syn).cuda()
    corr = torch.full((nw,), -1, dtype=torch.int64, device="cuda")
    flags = torch.zeros(len(code_of_shot), dtype=torch.uint8, device="cuda")
    iters = torch.zeros((len(code_of_shot), 2), dtype=torch.int16, device="cuda")
    outs = []
    if not graph:
        plan.decode_multi(cos, syn_t, so, corr, co, flags, iters)
        torch.cuda.synchronize()
        outs.append((corr.cpu().numpy().copy(), flags.cpu().numpy().copy(), iters.cpu().numpy().copy()))
    else:
        plan.capture_multi(cos, syn_t, so, corr, co, flags, iters)
        for _ in range(replays):
            corr.fill_(-1)
            flags.zero_()
            iters.zero_()
            torch.cuda.synchronize()
            plan.graph_launch()
            torch.cuda.synchronize()
            outs.append((corr.cpu().numpy().copy(), flags.cpu().numpy().copy(), iters.cpu().numpy().copy()))
            _ = torch.randn(1000, device="cuda").sum().item()   # unrelated eager work between replays
    return outs, co.cpu().numpy()


def _check_multi(P, prm, codes, per_code, out, corr_off):
    corr, flags, iters = out
    for i, c in enumerate(codes):
        idx, sh = per_code[i]
        nw = (c.n + 63) // 64
        for k, b in enumerate(idx):
            ref = oracle.decode(c, sh.syndromes[k:k + 1], oracle_params(prm, "channel"), precision="f32",
                                shot_offset=int(b), want_post=False)
            words = corr[corr_off[b]:corr_off[b] + nw].view(np.uint64)[None, :]
            np.testing.assert_array_equal(synth.unpack_bits(words, c.n), ref["ehat"])
            assert flags[b] == ref["flags"][0]
            np.testing.assert_array_equal(iters[b], ref["iters"][0])


def test_multi_code_single_launch_bit_exact(P):
    codes = [_small_hgp(j, nc, p=0.05) for j, nc in enumerate([16, 20, 24, 16])] + [synth.bb_code("bb144", p=0.05)]
    counts = [60, 50, 40, 30, 80]
    prm = P.Params(max_iter=(30, 30), alpha=0.625, seed=4)
    plan = P.Plan([P.Code.from_problem(c) for c in codes], prm, kernel=P.KERNEL_AUTO)
    code_of_shot, syn, per_code = _mixed_batch(P, codes, counts, 50)
    outs, corr_off = _run_multi(P, plan, codes, code_of_shot, syn)
    _check_multi(P, prm, codes, per_code, outs[0], corr_off)


# a circuit-level DEM (rows of 35: 64-bit check records, posteriors in slots sorted by column
# degree) in one launch with codes of rows of at most 32 edges (column order), all run by the
# 64-bit-record variant
def test_multi_code_mixed_record_widths_bit_exact(P):
    codes = [synth.bb_circuit_dem("bb72", 2, 0.003), synth.bb_code("bb144", p=0.05), _small_hgp(1, 20, p=0.05)]
    counts = [40, 60, 50]
    prm = P.Params(max_iter=(60, 60), alpha=0.625, seed=4)
    plan = P.Plan([P.Code.from_problem(c) for c in codes], prm, kernel=P.KERNEL_GROUP)
    code_of_shot, syn, per_code = _mixed_batch(P, codes, counts, 80)
    print("case multi-code circuit bb72 + bb144 + hgp20", flush=True)
    outs, corr_off = _run_multi(P, plan, codes, code_of_shot, syn)
    assert (outs[0][1] & 2).any(), "case must exercise DC"
    _check_multi(P, prm, codes, per_code, outs[0], corr_off)


def test_multi_code_graph_replays(P):
    codes = [_small_hgp(j, nc, p=0.05) for j, nc in enumerate([16, 24])]
    counts = [70, 50]
    prm = P.Params(max_iter=(30, 30), alpha=0.625, seed=4)
    plan = P.Plan([P.Code.from_problem(c) for c in codes], prm, kernel=P.KERNEL_GROUP)
    code_of_shot, syn, per_code = _mixed_batch(P, codes, counts, 60)
    eager, corr_off = _run_multi(P, plan, codes, code_of_shot, syn)
    replays, _ = _run_multi(P, plan, codes, code_of_shot, syn, graph=True, replays=3)
    for r in replays:
        for a, b in zip(r, eager[0]):
            np.testing.assert_array_equal(a, b)
    _check_multi(P, prm, codes, per_code, eager[0], corr_off)


def test_multi_code_out_of_range_index_is_flagged(P):
    """A code index outside [0, ncodes) is read on the device only: that shot is skipped
    with flags = FLAG_BAD_CODE, its correction words and iteration counts are left as they
    were, and every other shot of the batch decodes exactly as before."""
    import torch
    codes = [_small_hgp(j, nc, p=0.05) for j, nc in enumerate([16, 20])]
    counts = [50, 40]
    prm = P.Params(max_iter=(30, 30), alpha=0.625, seed=4)
    plan = P.Plan([P.Code.from_problem(c) for c in codes], prm, kernel=P.KERNEL_GROUP)
    code_of_shot, syn, per_code = _mixed_batch(P, codes, counts, 70)
    so, co, sw, nw = plan.multi_buffers(torch.from_numpy(code_of_shot).cuda())
    bad = {3: -1, 17: 2, 51: 1 << 30}
    cos_bad = code_of_shot.copy()
    for b, v in bad.items():
        cos_bad[b] = v
    print("case multi-code with out-of-range indices", bad, flush=True)
    corr = torch.full((nw,), -1, dtype=torch.int64, device="cuda")
    flags = torch.zeros(len(cos_bad), dtype=torch.uint8, device="cuda")
    iters = torch.full((len(cos_bad), 2), -7, dtype=torch.int16, device="cuda")
    plan.decode_multi(torch.from_numpy(cos_bad).cuda(), torch.from_numpy(syn).cuda(), so, corr, co, flags, iters)
    torch.cuda.synchronize()
    corr_h, flags_h, iters_h, co_h = (corr.cpu().numpy(), flags.cpu().numpy(), iters.cpu().numpy(),
                                      co.cpu().numpy())
    for b in bad:
        assert flags_h[b] == P.FLAG_BAD_CODE
        assert (iters_h[b] == -7).all()
        nwb = (codes[code_of_shot[b]].n + 63) // 64
        assert (corr_h[co_h[b]:co_h[b] + nwb] == -1).all()
    good = np.ones(len(cos_bad), bool)
    good[list(bad)] = False
    assert (flags_h[good] & P.FLAG_BAD_CODE == 0).all()
    for i, c in enumerate(codes):
        idx, sh = per_code[i]
        keep = [k for k, b in enumerate(idx) if good[b]]
        per_code[i] = (idx[keep], synth.ShotSet(sh.errors[keep], sh.syndromes[keep], sh.seed))
    _check_multi(P, prm, codes, per_code, (corr_h, flags_h, iters_h), co_h)
