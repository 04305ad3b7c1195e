"""The 48-beam batched job at full size, in the launch configuration bench.py times.

Every beam's chunk outputs from the persistent, graph-replayed batch must equal
plain per-beam calls bit for bit; plain calls of three beams (largest, smallest
and a middle one) are checked against the oracle on sampled DM rows of the
second time chunk, whose input is a view at a column offset of the whole
filterbank.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import oracle_table, sample_rows

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    return dd


def test_batch48_full_size(dd):
    import bench

    beams, chunkers, inputs, outputs, batches = bench.setup_batch48(dd, torch, synth,
                                                                    log=lambda m: print(m, flush=True))
    sizes = [b["n_chan"] * b["n_samp"] * b["n_dm"] for b in beams]
    order = np.argsort(sizes)
    checked = {int(order[-1]), int(order[0]), int(order[len(order) // 2])}
    for k, (idx, bt) in enumerate(batches):
        bt.run()
        torch.cuda.synchronize()
        print("chunk", k, "batched done", flush=True)
        for i in idx:
            c = chunkers[i]
            plan = c.plans[k]
            got = outputs[i][:, : plan.n_out].clone()
            plain = plan.forward(c.input_view(inputs[i], k))
            torch.cuda.synchronize()
            assert torch.equal(got, plain), ("beam", i, "chunk", k)
            if k == 1 and i in checked:
                b = beams[i]
                s = oracle_table(b)
                x = synth.gaussian_u8(b["n_chan"], b["n_samp"], b["seed"])
                rows = sample_rows(b["n_dm"], extra=3, seed=i)
                want = oracle.forward(x, "u8", b["n_samp"], s, rows=rows)
                t0 = c.spans[k][0]
                print("beam", i, "oracle rows", rows, "columns from", t0, flush=True)
                assert np.array_equal(plain[rows].cpu().numpy(), want[:, t0: t0 + plan.n_out])
                del x
            del got, plain
        print("chunk", k, "plain and oracle checks done", flush=True)
