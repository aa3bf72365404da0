"""GPU parity of the differentiable two-lobe fit: forward loss, lobe gradients and control-point
gradients (hand-written backward kernels) against the FP64 oracle's analytic gradient, at a
small fabric and at the full 2,000-fiber plain weave (levels 1-6, 128 directions).

Tolerances: the loss to 1e-5 relative (FP32 sums and FP32 profiles); the gradients to 1e-4
relative in norm over every lobe parameter and every control point.  Both sides take the same
direction values (the Fibonacci set rounded once to float32).  The backward pass differentiates
at FP64 level sums in FP64 arithmetic (a point's two segment-end terms, which nearly cancel along
a straight fiber, are added in FP64); what remains is the one FP32 rounding of each output."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _lattice_points(grid, pts):
    q = oracle.snap(grid, pts).astype(np.float64)
    return (np.asarray(grid.bmin) + q * (grid.extent / 2.0 ** 23)).astype(np.float32)


def _setup(vx, n_fibers, seed, lo=1, hi=6):
    import torch
    wl = synth.plain_weave(n_fibers=n_fibers, seed=seed)
    pts = _lattice_points(wl.grid, wl.pts)
    pd = torch.as_tensor(pts).cuda()
    od = torch.as_tensor(wl.offsets).cuda()
    plan = vx.FitPlan(wl.grid, pd, od, wl.radius, lo, hi, dirs=synth.fibonacci_dirs(128))
    params = vx.fit_init(plan, seed=4)
    return wl, pts, pd, plan, params


def _compare(vx, wl, pts, pd, plan, params, elementwise=False):
    import torch
    n_ref = oracle.fit_levels(wl.grid, pts, wl.offsets, wl.radius, 6)
    assert [int(x) for x in n_ref] == plan.counts
    loss = float(plan.forward(pd, params).item())
    L_all = np.concatenate([p.cpu().numpy() for p in params]).astype(np.float64)
    # both sides evaluate the same direction values (float32, exact in FP64)
    o_loss, _, o_dL, o_dp = oracle.fit_eval(wl.grid, pts, pts.astype(np.float64), wl.offsets, wl.radius, 1, 6, L_all,
                                            dirs=synth.fibonacci_dirs(128))
    say("loss", loss, o_loss)
    assert 1e-3 < o_loss < 1e9                      # a sane starting point, not uninitialised lobes
    assert abs(loss - o_loss) <= 1e-5 * o_loss
    dpts, dparams = plan.backward(torch.ones(1, device="cuda"), params)
    plan.check()
    g_dL = np.concatenate([d.cpu().numpy() for d in dparams]).astype(np.float64)
    g_dp = dpts.cpu().numpy().astype(np.float64)
    e_L = np.linalg.norm(g_dL - o_dL) / np.linalg.norm(o_dL)
    e_p = np.linalg.norm(g_dp - o_dp) / np.linalg.norm(o_dp)
    # per point, relative to the point's own gradient (floor: 1e-3 of the largest)
    pp = np.linalg.norm(g_dp - o_dp, axis=1) / np.maximum(np.linalg.norm(o_dp, axis=1),
                                                           1e-3 * np.linalg.norm(o_dp, axis=1).max())
    say("relative gradient errors: lobes %.3g, points %.3g (norm over all %d); worst point %.3g"
        % (e_L, e_p, len(g_dp), pp.max()))
    assert e_L <= 1e-4 and e_p <= 1e-4
    if elementwise:
        scale = np.abs(o_dL).max()
        bad = np.abs(g_dL - o_dL) > 1e-4 * np.abs(o_dL) + 1e-6 * scale
        say("lobe gradient entries outside 1e-4 relative (floor 1e-6 of the largest):", int(bad.sum()), "of",
            bad.size)
        assert not bad.any()


def test_fit_matches_oracle(vx):
    wl, pts, pd, plan, params = _setup(vx, 64, 14)
    say("case: fit on plain weave 64 fibers, levels 1..6, 128 directions")
    _compare(vx, wl, pts, pd, plan, params)


def test_fit_matches_oracle_full_weave(vx):
    """The differentiable-fit workload itself: 2,000 fibers x 256 segments at 1024^3, levels 1-6."""
    wl, pts, pd, plan, params = _setup(vx, 2000, 1)
    say("case: fit on the full plain weave (2000 fibers), levels 1..6, 128 directions;", sum(plan.counts[1:]),
        "fitted voxels")
    _compare(vx, wl, pts, pd, plan, params, elementwise=True)


def test_autograd_function_and_descent(vx):
    import torch
    wl, pts, pd, plan, params = _setup(vx, 32, 15)
    say("case: autograd wrapper, plain weave 32 fibers")
    P = [p.clone().requires_grad_(True) for p in params]
    X = pd.clone().requires_grad_(True)
    loss = vx.lobe_fit(plan, X, P)
    loss.backward()
    dpts, dparams = plan.backward(torch.ones(1, device="cuda"), [p.detach() for p in P])
    assert torch.equal(X.grad, dpts)
    for a, b in zip(P, dparams):
        assert torch.equal(a.grad, b)
    # a small gradient step on the lobes lowers the loss
    with torch.no_grad():
        Q = [p - 0.05 * p.grad for p in P]
    loss2 = vx.lobe_fit(plan, X.detach(), Q)
    l1, l2 = float(loss.detach()), float(loss2.detach())
    say("loss before/after one step", l1, l2)
    assert l2 < l1


def test_backward_after_another_forward_raises(vx):
    """Two live losses on one plan: the first one's backward must not see the second's state."""
    wl, pts, pd, plan, params = _setup(vx, 16, 16)
    say("case: two forwards on one plan, then the first backward")
    P = [p.clone().requires_grad_(True) for p in params]
    l1 = vx.lobe_fit(plan, pd, P)
    l2 = vx.lobe_fit(plan, pd, [p * 1.01 for p in P])
    with pytest.raises(RuntimeError):
        l1.backward()
    l2.backward()                                   # the latest one is still fine


def test_moved_points_are_reported_not_faulted(vx):
    """Points moved so that the fitted levels gain and change voxels: the parameters are bound to
    the calibration's voxels, so the call must report an error (never read or write past the
    parameter rows)."""
    import torch
    wl, pts, pd, plan, params = _setup(vx, 32, 17)
    say("case: fit with control points moved by 2.6 voxels after calibration")
    plan.forward(pd, params)
    moved = pd.clone()
    moved[:, 2] += 2.6 * wl.grid.extent / wl.grid.res     # every fiber moves up by 2.6 voxels
    moved[::7, 1] += 3.3 * wl.grid.extent / wl.grid.res
    with pytest.raises(vx.VxError) as e:
        plan.forward(moved, params)
    say("status", e.value.status)
    assert e.value.status in (2, 6)
    # the backward on the moved state is bounded too and reports the same
    with pytest.raises(vx.VxError):
        plan.backward(torch.ones(1, device="cuda"), params)
        plan.check()
    # and the original points still work
    plan.forward(pd, params)
    plan.backward(torch.ones(1, device="cuda"), params)
    plan.check()
