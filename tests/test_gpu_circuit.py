"""BP+DC on circuit-level detector error models of BB codes (Appendix C) on the
GPU against the float32 oracle (needs an MI355X).

H = H_DCM has rows of 35 edges, so the group kernel family runs it with its
64-bit per-check word (the lane family takes rows of at most 15 edges); the
plain family has no row limit for min-sum.  Bar: every output bit-exact with
the float32 oracle; at the benchmark size ([[144,12,12]], T = 12 rounds,
p = 0.001, 1000 + 1000 iterations, one launch of 20,000 shots) on sampled
blocks, plus properties on every shot."""
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


def _params(P, T):
    return P.Params(max_iter=T, alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=19)


@pytest.mark.parametrize("kernel", ["group", "plain"])
@pytest.mark.parametrize("name,rounds,p,shots,T", [("bb72", 3, 0.004, 600, (100, 100)),
                                                     ("bb72", 2, 0.002, 600, (300, 50))])
def test_circuit_dem_bit_exact_vs_float32_oracle(P, kernel, name, rounds, p, shots, T):
    code = synth.bb_circuit_dem(name, rounds, p)
    sh = synth.make_shots(code, shots, 8000 + shots + rounds)
    prm = _params(P, T)
    kid = P.KERNEL_GROUP if kernel == "group" else P.KERNEL_PLAIN
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
    print(f"case {name} T={rounds} p={p} shots={shots} kernel={kernel}", flush=True)
    g = gpu_decode(plan, code, sh.syndromes, shot_offset=11)
    ref = oracle.decode(code, sh.syndromes, oracle_params(prm, "channel"), precision="f32", shot_offset=11)
    assert ((ref["flags"] & 2) != 0).sum() > 10, "case must exercise DC"
    assert_bit_exact(g, ref, code.n)


# rows of 35 edges: the 64-bit-record variant keeps posteriors, priors and rows of D in slots
# sorted by column degree; the posterior second pass (its prior array in slot order, +inf on the
# cut) and intermittent soft DC (the nominees' priors raised in slot order), posteriors and cut
# masks included, bit-exact with the oracle
@pytest.mark.parametrize("mode", ["posterior", "soft"])
def test_circuit_dem_group_posterior_prior_and_soft_dc(P, mode):
    code = synth.bb_circuit_dem("bb72", 3, 0.004)
    sh = synth.make_shots(code, 400, 8400)
    if mode == "posterior":
        prm = P.Params(max_iter=(60, 60), alpha=0.625, second_pass_prior=P.PRIOR_POSTERIOR, seed=19)
    else:
        prm = P.Params(max_iter=(60, 60), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=19,
                       soft_period=5, soft_shift=0.5)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_GROUP)
    print(f"case circuit bb72 T=3 group {mode}", flush=True)
    g = gpu_decode(plan, code, sh.syndromes, shot_offset=5)
    ref = oracle.decode(code, sh.syndromes, oracle_params(prm, "posterior" if mode == "posterior" else "channel"),
                        precision="f32", shot_offset=5)
    assert ((ref["flags"] & 2) != 0).sum() > 10, "case must exercise DC"
    assert_bit_exact(g, ref, code.n)


def test_circuit_plan_choice(P):
    code = P.Code.from_problem(synth.bb_circuit_dem("bb72", 2, 0.002))
    prm = _params(P, (50, 50))
    assert P.Plan([code], prm, kernel=P.KERNEL_AUTO).info(0)["kernel"] == P.KERNEL_GROUP
    with pytest.raises(P.BpdcError):
        P.Plan([code], prm, kernel=P.KERNEL_LANE)
    # product-sum is refused on rows longer than 32 edges
    ps = P.Params(max_iter=(50, 50), alpha=1.0, second_pass_prior=P.PRIOR_CHANNEL, rule=P.RULE_PRODUCT_SUM)
    with pytest.raises(P.BpdcError):
        P.Plan([code], ps, kernel=P.KERNEL_PLAIN)


def test_circuit_full_size_batch_sampled(P):
    """[[144,12,12]], T = 12 rounds, p = 0.001, 1000 + 1000 iterations, 20,000 shots
    in one launch of the group kernel: sampled blocks against the float32 oracle."""
    import torch
    code = synth.bb_circuit_dem("bb144", 12, 0.001)
    B = 20_000
    sh = synth.make_shots(code, B, 2012)
    prm = _params(P, (1000, 1000))
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_GROUP)
    syn = torch.from_numpy(synth.pack_bits(sh.syndromes).view(np.int64)).cuda()
    print("case bb144 circuit T=12 p=0.001 B=20000 group", flush=True)
    out = plan.decode(syn, want_cut=True, want_iters=True)
    torch.cuda.synchronize()
    corr = synth.unpack_bits(out["corr"].cpu().numpy().view(np.uint64), code.n)
    flags = out["flags"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    cut = synth.unpack_bits(out["cut"].cpu().numpy().view(np.uint64), code.n)
    for lo in (0, 9_950, 19_950):
        hi = lo + 50
        ref = oracle.decode(code, sh.syndromes[lo:hi], oracle_params(prm, "channel"), precision="f32",
                            shot_offset=lo, want_post=False)
        np.testing.assert_array_equal(corr[lo:hi], ref["ehat"])
        np.testing.assert_array_equal(flags[lo:hi], ref["flags"])
        np.testing.assert_array_equal(iters[lo:hi], ref["iters"])
        np.testing.assert_array_equal(cut[lo:hi], ref["cut"])
    conv = (flags & 1) != 0
    assert (synth.syndromes_of(corr[conv], code.H) == sh.syndromes[conv]).all()
    dc = (flags & 2) != 0
    assert (iters[dc, 0] == 1000).all() and (iters[~dc, 1] == 0).all()
    assert not (corr & cut).any()
    # one cut column per row of D at most
    assert (cut[dc].sum(1) <= code.D.rows).all() and (cut[dc].sum(1) > 0).all()
