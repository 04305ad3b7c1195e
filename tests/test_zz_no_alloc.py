"""dd_execute_noalloc (tables in the library's static device area, nothing allocated)
against dd_execute of the same plan: identical outputs, over consecutive calls whose
plans differ (the area keeps only the last call's tables), the second one smaller,
for 8-bit (both staging forms), 4-bit, 16-bit and float input."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    assert torch.cuda.is_available()
    return dd


def _desc(dtype, n_chan, n_samp, n_dm, step):
    return dict(n_chan=n_chan, n_samp=n_samp, dtype=dtype, f_high=1500.0, chan_bw=300.0 / n_chan, t_samp=64e-6,
                dm_start=0.0, dm_step=step, n_dm=n_dm)


def _input(dtype, n_chan, n_samp, seed):
    if dtype == "u8":
        return synth.gaussian_u8(n_chan, n_samp, seed)
    if dtype == "u4":
        return synth.uniform_u4_packed(n_chan, n_samp, seed)
    if dtype == "u16":
        return synth.gaussian_u16(n_chan, n_samp, seed)
    return synth.normal_f32(n_chan, n_samp, seed)


def _both(dd, desc, seed, shape=None):
    """(dd_execute output, dd_execute_noalloc output) of one plan on one seeded input."""
    bound = dd.Plan(**desc)
    free = dd.Plan(**desc, bind=False)  # never bound: its tables only ever live in the static area
    if shape is not None:
        bound.set_tiles(0, shape, 2)
        free.set_tiles(0, shape, 2)
    assert bound.tiles(0) == free.tiles(0)
    x = torch.from_numpy(_input(desc["dtype"], desc["n_chan"], desc["n_samp"], seed)).cuda()
    want = bound.forward(x)
    out = torch.full((free.n_dm, free.out_pitch), float("nan"), device="cuda")
    got = free.forward_noalloc(x, out)
    torch.cuda.synchronize()
    return want.cpu().numpy(), got.cpu().numpy()


def _shape_index(dd, desc, segs):
    """First compiled shape of the plan with the requested staging form (0 ring, > 0 phase loads)."""
    p = dd.Plan(**desc, bind=False)
    for s in range(p.n_shapes):
        try:
            p.set_tiles(0, s, 2)
        except dd.DDError:
            continue
        t = p.tiles(0)
        if t["row_block"] > 0 and (t["segs"] > 0) == (segs > 0):
            return s
    pytest.skip("no shape of that staging form holds the plan")


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_noalloc_matches_execute_two_calls(dtype, dd):
    big = _desc(dtype, 256, 40000, 96, 1.0)
    small = _desc(dtype, 64, 9024, 40, 2.0)
    tol = 0.0  # same kernels, same fixed summation order: identical bits for every input type
    for desc, seed in ((big, 11), (small, 12), (big, 13)):
        want, got = _both(dd, desc, seed)
        assert got.shape == want.shape
        assert np.isfinite(got).all()
        assert np.abs(got - want).max() <= tol, (dtype, desc["n_chan"], desc["n_samp"])


def test_noalloc_both_8bit_staging_forms_and_direct(dd):
    desc = _desc("u8", 200, 30000, 80, 1.0)
    small = _desc("u8", 48, 8000, 33, 1.5)
    for segs in (0, 1):
        for d, seed in ((desc, 21), (small, 22)):
            s = _shape_index(dd, d, segs)
            want, got = _both(dd, d, seed, shape=s)
            assert np.array_equal(got, want), ("segs", segs, d["n_chan"])
    # a direct-read shape: its tables are the plain shift table
    p = dd.Plan(**desc, bind=False)
    direct = []
    for s in range(p.n_shapes):
        try:
            p.set_tiles(0, s, 0)
        except dd.DDError:
            continue
        if p.tiles(0)["row_block"] == 0:
            direct.append(s)
    assert direct
    for d, seed in ((desc, 23), (small, 24)):
        want, got = _both(dd, d, seed, shape=direct[0])
        assert np.array_equal(got, want)
    # 4-bit plans read directly by default; their staged forms use the static area too
    d4 = _desc("u4", 200, 30016, 80, 1.0)
    for segs in (0, 1):
        want, got = _both(dd, d4, 25 + segs, shape=_shape_index(dd, d4, segs))
        assert np.array_equal(got, want), ("u4 segs", segs)


def test_noalloc_refuses_tables_beyond_the_static_area(dd):
    desc = _desc("u8", 8192, 1 << 17, 4000, 0.5)  # headline-sized tables, far above 32 MiB
    p = dd.Plan(**desc, bind=False)
    assert p.info.dev_table_bytes > 32 << 20
    x = torch.zeros((p.n_chan, p.in_row_elems), dtype=torch.uint8, device="cuda")
    out = torch.empty((p.n_dm, p.out_pitch), dtype=torch.float32, device="cuda")
    with pytest.raises(dd.DDError) as e:
        p.forward_noalloc(x, out)
    assert e.value.name == "DD_ERR_RANGE"
