"""The allocation-free likelihood entry point (smcgw_loglike_grad_noalloc) against smcgw_loglike_grad.

Two calls in a row, the second with fewer particles, each in both precisions: the outputs equal the
allocating entry point's bit for bit (same kernels, scratch in the fixed device array instead of the
context's).  A batch beyond the array's capacity is refused on the host before anything is queued.
"""
import numpy as np
import pytest
import torch

from paper_2601_02336_amd import synth

from helpers import event

pytestmark = pytest.mark.gpu


def test_noalloc_equals_loglike_grad():
    from paper_2601_02336_amd import smcgw
    ev = event(synth.SPEC_8S)   # 3 detectors, 8033 bins, 11 parameters
    b = synth.gw_prior_for(ev)
    c = smcgw.Context(0)
    c.add_event(ev)
    for P in (3000, 700):
        x = torch.tensor(synth.prior_draw(np.random.default_rng(P), P, b), device="cuda")
        for prec in (smcgw.MIXED, smcgw.PLAIN_FP64):
            ll_ref, g_ref = c.loglike_grad(x, precision=prec)
            ll = torch.full((P,), float("nan"), dtype=torch.float64, device="cuda")
            g = torch.full((P, 11), float("nan"), dtype=torch.float64, device="cuda")
            assert c.loglike_grad_noalloc(x, ll, g, precision=prec) == smcgw.OK
            torch.cuda.synchronize()
            print(f"P={P} precision={prec}: max |dlogL| {float((ll - ll_ref).abs().max()):.1e}", flush=True)
            assert torch.equal(ll, ll_ref) and torch.equal(g, g_ref)
            ll2 = torch.full((P,), float("nan"), dtype=torch.float64, device="cuda")
            assert c.loglike_grad_noalloc(x, ll2, None, precision=prec) == smcgw.OK   # forward only
            torch.cuda.synchronize()
            assert torch.equal(ll2, ll_ref)
    n = smcgw.NOALLOC_MAX_P + 1
    big = torch.zeros((n, 11), dtype=torch.float64, device="cuda")
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert c.loglike_grad_noalloc(big, out, None) == smcgw.ERR_SHAPE
    c.close()
