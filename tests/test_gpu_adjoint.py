"""GPU adjoint (gather form) and autograd against the oracle's scatter-form transpose.

Checks: element parity within the FP32 bound, exact zeros where no output
reads a sample, the FP64 dot-product test <Ax, y> = <x, A^T y> at rel <= 1e-6
on the full gradient workload, and central finite differences of
loss = sum (A x - target)^2 through torch.autograd.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import oracle_table, plan_for

pytestmark = pytest.mark.gpu

FD_TOL = 2e-3


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    return dd


ADJ_CASES = [  # (n_chan, n_samp, n_dm)
    (1, 2000, 3), (7, 3001, 5), (40, 9000, 33), (100, 20000, 64), (300, 6000, 100), (33, 70000, 7),
]


@pytest.mark.parametrize("case", ADJ_CASES)
def test_adjoint_matches_scatter_oracle(dd, case):
    n_chan, n_samp, n_dm = case
    rng = np.random.default_rng(n_chan + 7 * n_dm)
    f_high = 1500.0
    bw = 300.0 / n_chan if n_chan > 1 else 1.0
    t_samp = 128e-6
    k = 1 / (f_high - (n_chan - 1) * bw) ** 2 - 1 / f_high**2
    dm_max = 0.5 * n_samp * t_samp / (4.148808e3 * k) if k > 0 else 1.0
    cfg = dict(dtype="f32", n_chan=n_chan, n_samp=n_samp, f_high=f_high, chan_bw=bw, t_samp=t_samp,
               dm_start=0.1 * dm_max, dm_step=0.9 * dm_max / max(n_dm - 1, 1), n_dm=n_dm)
    s = oracle_table(cfg)
    n_out = oracle.n_out_for(s, n_samp)
    pitch = (n_samp + 3) // 4 * 4
    plan = plan_for(dd, cfg, in_pitch_bytes=pitch * 4)
    y = rng.standard_normal((n_dm, n_out)).astype(np.float32)
    g = plan.adjoint(torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    got = g.cpu().numpy().astype(np.float64)
    want = oracle.adjoint(y, n_chan, n_samp, s)
    # the bound: 1e-5 * sum of |terms| feeding each sample
    ab = oracle.adjoint(np.abs(y), n_chan, n_samp, s)
    assert (np.abs(got - want) <= 1e-5 * ab).all()
    assert (got[ab == 0] == 0).all()  # samples no output reads are exact zeros


def test_dot_product_full_workload(dd):
    """<A x, y> = <x, A^T y> in FP64 on 1024 ch x 2^17 x 1024 DMs, N(0,1) inputs: rel <= 1e-6."""
    cfg = synth.CONFIGS["grad_f32"]
    plan = plan_for(dd, cfg)
    x = torch.from_numpy(synth.normal_f32(cfg["n_chan"], cfg["n_samp"], cfg["seed"])).cuda()
    gen = torch.Generator(device="cpu").manual_seed(cfg["target_seed"])
    y = torch.randn((cfg["n_dm"], plan.out_pitch), generator=gen).cuda()
    y[:, plan.n_out:] = 0
    ax = plan.forward(x)
    aty = plan.adjoint(y)
    lhs = (ax.double() * y[:, : plan.n_out].double()).sum().item()
    rhs = (x[:, : cfg["n_samp"]].double() * aty.double()).sum().item()
    rel = abs(lhs - rhs) / max(abs(lhs), abs(rhs))
    assert rel <= 1e-6, rel


def test_dot_product_exact_small_integers(dd):
    """With small integers every float32 sum is exact, so the dot test holds exactly."""
    cfg = dict(dtype="f32", n_chan=96, n_samp=6000, f_high=1500.0, chan_bw=300.0 / 96, t_samp=128e-6,
               dm_start=0.0, dm_step=4.0, n_dm=48)
    plan = plan_for(dd, cfg)
    rng = np.random.default_rng(9)
    x = torch.from_numpy(rng.integers(-15, 16, (96, 6000)).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.integers(-3, 4, (48, plan.out_pitch)).astype(np.float32)).cuda()
    ax = plan.forward(x)
    aty = plan.adjoint(y)
    lhs = (ax.double() * y[:, : plan.n_out].double()).sum().item()
    rhs = (x.double() * aty.double()).sum().item()
    assert lhs == rhs


def test_autograd_central_differences(dd):
    """Gradient of loss = sum (A x - target)^2 through DedisperseFn vs central differences.

    The loss is exactly quadratic, so with h = 0.5 the central difference has no
    truncation error; the difference of the two losses is taken only over the
    outputs the perturbed sample feeds (the rest cancel exactly).  What remains
    is the float32 rounding of the two forward evaluations: the difference
    quotient picks up sum_d a_d (delta+_d - delta-_d) / h, about 1.5e-4 of the
    gradient (one sigma) for 1024 N(0,1) channels, so FD_TOL is ~10 sigma.  The
    gradient itself is held to 1e-4 against Eq. 3 evaluated in FP64, and the
    exact version with small integers is test_autograd_exact_small_integers.
    """
    cfg = synth.CONFIGS["grad_f32"]
    plan = plan_for(dd, cfg)
    x0 = torch.from_numpy(synth.normal_f32(cfg["n_chan"], cfg["n_samp"], cfg["seed"])).cuda()
    gen = torch.Generator(device="cpu").manual_seed(cfg["target_seed"])
    target = torch.randn((cfg["n_dm"], plan.n_out), generator=gen).cuda()
    x = x0.clone().requires_grad_(True)
    out = dd.DedisperseFn.apply(x, plan)
    loss = ((out.double() - target.double()) ** 2).sum()
    loss.backward()
    grad = x.grad
    s = plan.shift
    rng = np.random.default_rng(cfg["fd_seed"])
    picks = [(int(c), int(t)) for c, t in zip(rng.integers(0, cfg["n_chan"], 62), rng.integers(0, cfg["n_samp"], 62))]
    picks += [(0, cfg["n_samp"] - 1), (0, plan.n_out)]  # channel 0 never delays: these feed no output
    h = 0.5
    xh = x0.cpu().numpy().astype(np.float64)
    th = target.cpu().numpy().astype(np.float64)
    chans = np.arange(cfg["n_chan"])
    for c, t in picks:
        xp = x0.clone()
        xp[c, t] += h
        xm = x0.clone()
        xm[c, t] -= h
        op = plan.forward(xp)
        om = plan.forward(xm)
        u = t - s[:, c].astype(np.int64)  # output sample each DM row reads this input at
        dsel = np.nonzero((u >= 0) & (u < plan.n_out))[0]
        dd_ = torch.from_numpy(dsel).cuda()
        uu_ = torch.from_numpy(u[dsel]).cuda()
        lp = ((op[dd_, uu_].double() - target[dd_, uu_].double()) ** 2).sum()
        lm = ((om[dd_, uu_].double() - target[dd_, uu_].double()) ** 2).sum()
        fd = ((lp - lm) / (2 * h)).item()
        g = grad[c, t].item()
        assert abs(fd - g) <= FD_TOL * max(1.0, abs(fd)), (c, t, fd, g)
        # Eq. 3 evaluated directly in FP64 at the outputs this sample feeds: 2 * sum_d (S - target)
        if len(dsel):
            sv = xh[chans[None, :], u[dsel][:, None] + s[dsel, :]].sum(axis=1)
            ref = 2.0 * float((sv - th[dsel, u[dsel]]).sum())
        else:
            ref = 0.0
        assert abs(ref - g) <= 1e-4 * max(1.0, abs(ref)), (c, t, ref, g)
    assert grad[0, cfg["n_samp"] - 1].item() == 0.0 and grad[0, plan.n_out].item() == 0.0


def test_autograd_exact_small_integers(dd):
    """Integer x in [-3, 3], integer target, h = 1: every float32 sum in the forward,
    the residual and the adjoint is exact, so central differences equal the
    autograd gradient exactly."""
    cfg = dict(dtype="f32", n_chan=1024, n_samp=1 << 14, f_high=1500.0, chan_bw=300.0 / 1024, t_samp=128e-6,
               dm_start=0.0, dm_step=0.5, n_dm=256)
    plan = plan_for(dd, cfg)
    rng = np.random.default_rng(17)
    x0 = torch.from_numpy(rng.integers(-3, 4, (1024, 1 << 14)).astype(np.float32)).cuda()
    target = torch.from_numpy(rng.integers(-3, 4, (256, plan.n_out)).astype(np.float32)).cuda()
    x = x0.clone().requires_grad_(True)
    out = dd.DedisperseFn.apply(x, plan)
    ((out.double() - target.double()) ** 2).sum().backward()
    grad = x.grad
    s = plan.shift
    for c, t in zip(rng.integers(0, 1024, 64), rng.integers(0, 1 << 14, 64)):
        c, t = int(c), int(t)
        xp = x0.clone()
        xp[c, t] += 1.0
        xm = x0.clone()
        xm[c, t] -= 1.0
        op, om = plan.forward(xp), plan.forward(xm)
        u = t - s[:, c].astype(np.int64)
        dsel = np.nonzero((u >= 0) & (u < plan.n_out))[0]
        dd_, uu_ = torch.from_numpy(dsel).cuda(), torch.from_numpy(u[dsel]).cuda()
        lp = ((op[dd_, uu_].double() - target[dd_, uu_].double()) ** 2).sum()
        lm = ((om[dd_, uu_].double() - target[dd_, uu_].double()) ** 2).sum()
        assert ((lp - lm) / 2.0).item() == grad[c, t].item(), (c, t)


def test_adjoint_full_workload_sampled_channels(dd):
    """The adjoint at the full differentiation size (1024 ch x 2^17 x 1024 DMs) against the
    oracle's scatter form, element by element on sampled channels (every time sample of each):
    the oracle runs on the shift sub-table of those channels, which includes the lowest channel,
    so its N_out is the plan's.  y is N(0,1) and passed with row pitch n_out (not a multiple of 4),
    the layout a gradient tensor arrives in."""
    cfg = synth.CONFIGS["grad_f32"]
    plan = plan_for(dd, cfg)
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    assert plan.n_out % 4 != 0
    gen = torch.Generator(device="cpu").manual_seed(cfg["target_seed"] + 1)
    y = torch.randn((cfg["n_dm"], plan.n_out), generator=gen)
    g = plan.adjoint(y.cuda())
    torch.cuda.synchronize()
    s = plan.shift
    rng = np.random.default_rng(23)
    chans = sorted({0, 1, n_chan // 2, n_chan - 2, n_chan - 1} | {int(c) for c in rng.integers(0, n_chan, 11)})
    sub = np.ascontiguousarray(s[:, chans])
    yn = y.numpy()
    want = oracle.adjoint(yn, len(chans), n_samp, sub)
    ab = oracle.adjoint(np.abs(yn), len(chans), n_samp, sub)
    got = g[chans].cpu().numpy().astype(np.float64)
    err = np.abs(got - want)
    assert (err <= 1e-5 * ab).all(), float((err / np.maximum(ab, 1e-30)).max())
    assert (got[ab == 0] == 0).all()


def test_autograd_pitched_view_and_no_gradient_copy(dd):
    """DedisperseFn on a view of the first n_samp columns of a pitched buffer and on the whole
    buffer: the gradient has the input's shape, equals the adjoint of 2 (A x - target), is zero
    on columns past n_samp, and the incoming gradient reaches the adjoint without a copy."""
    n_chan, n_samp, n_dm = 96, 6001, 40
    cfg = dict(dtype="f32", n_chan=n_chan, n_samp=n_samp, f_high=1500.0, chan_bw=300.0 / n_chan, t_samp=128e-6,
               dm_start=0.0, dm_step=3.0, n_dm=n_dm)
    pitch = 6016  # floats; 64 bytes of row padding past the last whole 16-byte chunk
    plan = plan_for(dd, cfg, in_pitch_bytes=4 * pitch)
    assert plan.n_out % 4 != 0
    rng = np.random.default_rng(31)
    base = torch.from_numpy(rng.integers(-8, 9, (n_chan, pitch)).astype(np.float32)).cuda()
    target = torch.from_numpy(rng.integers(-8, 9, (n_dm, plan.n_out)).astype(np.float32)).cuda()
    seen = {}
    orig = plan.adjoint

    def spy(y, out=None, stream=None):
        seen["y"] = y.data_ptr()
        return orig(y, out=out, stream=stream)
    plan.adjoint = spy
    try:
        for cols in (n_samp, pitch):
            leaf = base.clone().requires_grad_(True)
            x = leaf[:, :cols]
            out = dd.DedisperseFn.apply(x, plan)
            out.register_hook(lambda g: seen.__setitem__("grad_out", g.data_ptr()))
            ((out - target) ** 2).sum().backward()
            assert seen["y"] == seen["grad_out"], "the incoming gradient was copied"
            want = orig(2.0 * (plan.forward(base) - target)).cpu()  # exact: small integers
            got = leaf.grad.cpu()
            assert got.shape == (n_chan, pitch)
            assert torch.equal(got[:, :n_samp], want)
            assert (got[:, n_samp:] == 0).all()
    finally:
        plan.adjoint = orig
