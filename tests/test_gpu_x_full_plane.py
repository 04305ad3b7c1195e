"""Every output of the headline workload (8192 ch u8 x 2^20 x 4000 DMs), not just sampled rows.

The oracle's plain loops would need about 8 minutes of host time for the whole
3.3e13-add plane, so the rows are recomputed on the host by the tiled CPU
implementation of Algorithm 2 (libdd_cpu.so), which shares no code with the
GPU kernels and is itself checked bit for bit against the oracle
(test_cpu_tiled.py); the oracle still checks sampled rows directly
(test_gpu_forward.py).  Blocks of 500 DM rows keep host memory bounded.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import plan_for

pytestmark = pytest.mark.gpu


def test_headline_full_plane_bit_exact():
    import paper_2311_05341_amd as dd
    from paper_2311_05341_amd import cpu_tiled

    cfg = synth.CONFIGS["headline"]
    s = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], cfg["dm_start"],
                           cfg["dm_step"], cfg["n_dm"])
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    print("full plane: generating input", flush=True)
    xd = torch.empty((n_chan, n_samp), dtype=torch.uint8, device="cuda")
    table = torch.from_numpy(synth.gaussian_table()).cuda()
    synth.gaussian_u8_device(xd.data_ptr(), n_chan, n_samp, n_samp, cfg["seed"], table.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    xh = synth.gaussian_u8(n_chan, n_samp, cfg["seed"])
    plan = plan_for(dd, cfg)
    assert np.array_equal(plan.shift, s)
    out = plan.forward(xd)
    torch.cuda.synchronize()
    for c in (0, 8191):
        assert torch.equal(xd[c].cpu(), torch.from_numpy(xh[c]))
    n_out = plan.n_out
    for d0 in range(0, cfg["n_dm"], 500):
        print("full plane: rows %d.." % d0, flush=True)
        want = cpu_tiled.forward_u8(xh, s[d0:d0 + 500], n_out)
        assert np.array_equal(out[d0:d0 + 500].cpu().numpy(), want), d0
