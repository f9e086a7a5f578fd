"""The allocation-free evaluation (gst_loglik_noalloc) against gst_loglik.

Both run the same kernels over the same grid; only the scratch differs (a
static device array instead of the context's workspace), so objective,
probabilities and gradient must be equal bit for bit.  Two calls in a row, the
second on a smaller list, each compared with gst_loglik on the same inputs;
the device's free memory does not change across the calls; refused inputs
are refused before anything runs."""
import sys

import numpy as np
import pytest

from paper_2008_13490_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_13490_amd import api
    return api, api.Context(0), torch


def _inputs(api, torch, kind, S, lmax, seed):
    w = W.random_workload(kind, S, lmax, seed)
    gs = api.DeviceGateSet.from_numpy(w.model.n_qubits, w.model.rho, w.model.effects, w.model.gates)
    seqs = api.DeviceSeqs.from_numpy(w.seqs.offsets, w.seqs.gates)
    counts = torch.as_tensor(w.counts, device="cuda")
    return w, gs, seqs, counts


def test_noalloc_equals_loglik_on_two_calls(gpu):
    api, ctx, torch = gpu
    cases = [("2q", 3000, 120, 61), ("2q", 700, 40, 62), ("1q", 900, 200, 63)]
    for kind, S, lmax, seed in cases:
        w, gs, seqs, counts = _inputs(api, torch, kind, S, lmax, seed)
        say(f"[noalloc] {kind} S={S} max_len={seqs.max_len}")
        ref = ctx.loglik(gs, seqs, counts, want_probs=True, want_grad=True)
        out = (torch.empty_like(ref[0]), torch.empty_like(ref[1]), torch.empty_like(ref[2]))
        ctx.loglik_noalloc(gs, seqs, counts, out)      # first call on this input (module loaded before)
        ctx.sync()
        free0 = torch.cuda.mem_get_info()[0]
        ctx.loglik_noalloc(gs, seqs, counts, out)
        ctx.sync()
        assert torch.cuda.mem_get_info()[0] == free0
        for x, y in zip(ref, out):
            assert torch.equal(x, y)


def test_noalloc_refuses_what_it_cannot_do(gpu):
    from paper_2008_13490_amd import _lib
    api, ctx, torch = gpu
    w, gs, seqs, counts = _inputs(api, torch, "2q", 50, 10, 64)
    out = (torch.empty(1, dtype=torch.float64, device="cuda"), None, None)
    unknown = api.DeviceSeqs(seqs.offsets, seqs.gates, -1)
    with pytest.raises(_lib.GSTError) as e:
        ctx.loglik_noalloc(gs, unknown, counts, out)
    assert e.value.code == _lib.GST_EINVAL
    g3 = W.random_workload("3q", 20, 10, 65)
    gs3 = api.DeviceGateSet.from_numpy(3, g3.model.rho, g3.model.effects, g3.model.gates)
    s3 = api.DeviceSeqs.from_numpy(g3.seqs.offsets, g3.seqs.gates)
    with pytest.raises(_lib.GSTError) as e:
        ctx.loglik_noalloc(gs3, s3, torch.as_tensor(g3.counts, device="cuda"), out)
    assert e.value.code == _lib.GST_EINVAL
    # a list whose checkpoints exceed the array: refused before anything is launched
    big = api.DeviceSeqs(seqs.offsets, seqs.gates, 1 << 20)
    with pytest.raises(_lib.GSTError) as e:
        ctx.loglik_noalloc(gs, big, counts, (out[0], None, torch.empty(1616 + 512, dtype=torch.float64,
                                                                      device="cuda")))
    assert e.value.code == _lib.GST_EINVAL and "scratch" in str(e.value)
