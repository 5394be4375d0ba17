"""Error paths of the C ABI on a GPU, driven from the host: the library's
fault-injection hook reports one checked HIP status as failed, so every
phase of a call (set-up, copies, launches, read-back) takes its error path
while nothing fails on the device."""

import numpy as np
import pytest

from paper_1304_2272_amd import binding, synth

pytestmark = pytest.mark.gpu

GWAS_E_HIP, GWAS_E_STATE = 5, 7


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    binding.load()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_injected_failure_poisons_only_its_context(precision):
    # A block of 700 SNPs in sub-blocks of 256: three sub-blocks, each with
    # its copies, product, cross products and solves.  Failing the k-th
    # checked status for growing k walks the failure through the call; each
    # time the call reports GWAS_E_HIP, the context refuses later calls, it
    # can still be freed, and a fresh context then gives the same bits as
    # before.
    n, p, m, seed = 300, 4, 700, 53
    prob = synth.make_problem(n, p, seed)
    XR = synth.snp_block(n, seed, 0, m, dtype=np.int8)
    kw = dict(precision=precision, x_dtype="i8", dev_block=256)
    with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], **kw) as ctx:
        b_ref, v_ref, i_ref = ctx.stream_block(XR)
    failed = 0
    for k in (1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233):
        _say(f"{precision}: failing checked status {k}")
        ctx = binding.GwasContext(prob["M"], prob["XL"], prob["Y"], **kw)
        try:
            ctx.inject_fault(k)
            try:
                out = ctx.stream_block(XR)
            except binding.GwasError as e:
                assert e.code == GWAS_E_HIP and "(injected)" in str(e), str(e)
                failed += 1
                with pytest.raises(binding.GwasError) as again:
                    ctx.stream_block(XR)
                assert again.value.code == GWAS_E_STATE
            else:
                # the call checks fewer statuses than k: it completed normally
                assert np.array_equal(out[0], b_ref) and np.array_equal(out[1], v_ref)
        finally:
            ctx.close()
    assert failed >= 6
    with binding.GwasContext(prob["M"], prob["XL"], prob["Y"], **kw) as ctx:
        b, v, i = ctx.stream_block(XR)
    assert np.array_equal(b, b_ref) and np.array_equal(v, v_ref) and np.array_equal(i, i_ref)


def test_injected_failure_in_a_group_leaves_other_contexts_usable():
    # The first context of a grouped call takes the failure; the second one,
    # whose copies the call had queued too, stays usable and exact.
    p, m = 4, 600
    probs = [synth.make_problem(n, p, 60 + i) for i, n in enumerate((400, 700))]
    XRs = [synth.snp_block(pr["n"], 61, 0, m, dtype=np.int8, cohort=i) for i, pr in enumerate(probs)]
    kw = dict(precision="fp32", x_dtype="i8", dev_block=256)
    refs = []
    for pr, X in zip(probs, XRs):
        with binding.GwasContext(pr["M"], pr["XL"], pr["Y"], **kw) as ctx:
            refs.append(ctx.stream_block(X)[0])
    for k in (4, 30, 120):
        _say(f"group: failing checked status {k}")
        ctxs = [binding.GwasContext(pr["M"], pr["XL"], pr["Y"], **kw) for pr in probs]
        try:
            ctxs[0].inject_fault(k)
            try:
                binding.stream_group(ctxs, XRs)
            except binding.GwasError as e:
                assert e.code == GWAS_E_HIP and "(injected)" in str(e), str(e)
            b1 = ctxs[1].stream_block(XRs[1])[0]
            assert np.array_equal(b1, refs[1])
        finally:
            for c in ctxs:
                c.close()
