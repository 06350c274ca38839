"""GPU tests of the on-device accuracy metrics (sne_accuracy): e_A and e_P of
eq. ea_ep against the FP64 oracle and against closed forms.

Tolerance.  The kernel forms each angle from the same FP32 inputs as the
oracle, in FP32 (cross and dot products of unit vectors, atan2): about 1e-7
rad, i.e. < 1e-5 degrees per pixel, so |e_A(GPU) - e_A(oracle)| <= 1e-4
degrees.  A pixel's e_P vote may differ only if its angle lies within that
distance of the threshold; m is exact."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2005_08165_amd import scenes as S
from paper_2005_08165_amd import sne

pytestmark = pytest.mark.gpu

TOL_DEG = 1e-4


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check(ctx, est, gt, mask, phis):
    """GPU metrics against the oracle on the very same values."""
    eA, eP, m = ctx.accuracy(est, gt, mask, phis)
    n64 = est.double().cpu().numpy()
    g64 = gt.double().cpu().numpy()
    mk = None if mask is None else mask.cpu().numpy()
    oA, oP, om = oracle.accuracy(n64, g64, mk, phis)
    assert m == om
    assert abs(eA - oA) <= TOL_DEG, (eA, oA)
    if m:
        psi = oracle.angular_error_deg(np.moveaxis(n64, -3, 0), np.moveaxis(g64, -3, 0))
        if mk is not None:
            psi = psi[mk != 0]
        for p, a, b in zip(phis, eP, oP):
            near = int(np.sum(np.abs(psi - p) <= TOL_DEG))
            assert abs(a - b) * m <= near + 1e-6, (p, a, b, near)
    return eA, eP, m


def _rotated(seed, shape, theta_deg):
    """Unit ground truth and vectors at the given angles from it (scaled)."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    g = rng.normal(size=(n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    u = np.cross(g, rng.normal(size=(n, 3)))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    t = np.radians(theta_deg.reshape(-1))[:, None]
    v = (np.cos(t) * g + np.sin(t) * u) * rng.uniform(0.5, 2.0, size=(n, 1))
    to = lambda a: torch.from_numpy(
        np.moveaxis(a.reshape(shape + (3,)), -1, -3).copy()).float().cuda()
    return to(v), to(g)


@pytest.mark.parametrize("shape", [(3, 67, 131), (2, 64, 96)])
@pytest.mark.parametrize("out", ["f32", "f16"])
def test_accuracy_closed_form_and_oracle(out, shape):
    """Vectors at known angles from the ground truth, frames of 67x131 (one
    pixel at a time, ragged against the 256-thread blocks) and of 64x96
    (groups of four pixels), a random mask: the GPU metrics match the oracle
    within the tolerance and e_A the mean of the angles."""
    rng = np.random.default_rng(21)
    theta = rng.uniform(0.0, 180.0, size=shape)
    est, gt = _rotated(22, shape, theta)
    if out == "f16":
        est = est.half()
    mask = torch.from_numpy(rng.integers(0, 2, size=shape).astype(np.uint8)).cuda()
    ctx = sne.Context(0)
    phis = (5.0, 11.25, 22.5, 30.0, 90.0, 179.0)
    eA, eP, m = _check(ctx, est, gt, mask, phis)
    keep = mask.cpu().numpy() != 0
    assert m == int(keep.sum())
    if out == "f32":  # the FP32 rounding of the vectors moves angles by ~1e-5 degrees
        assert abs(eA - theta[keep].mean()) <= TOL_DEG


@pytest.mark.parametrize("out", ["f32", "f16"])
def test_accuracy_of_estimated_normals(out):
    """The indoor scene's estimate (FD-mean) against its analytic normals:
    the use the metrics are for."""
    fr = S.make_indoor(0)
    gt = fr.gt.float().cuda().contiguous()
    n, msk = sne.estimate(fr.raw.cuda(), fr.cam.as_tuple(), "depth_f32", "fd", "mean", out)
    ctx = sne.Context(0)
    eA, eP, m = _check(ctx, n.contiguous(), gt, msk, (1.0, 5.0, 11.25))
    say("indoor FD-mean %s: e_A %.4f deg, e_P %s, m %d" % (out, eA, eP, m))
    assert m > 0.5 * 480 * 640 and eA < 5.0


def test_accuracy_without_mask_and_empty():
    shape = (2, 40, 50)
    theta = np.full(shape, 30.0)
    est, gt = _rotated(23, shape, theta)
    ctx = sne.Context(0)
    eA, eP, m = _check(ctx, est, gt, None, (29.0, 31.0))
    assert m == 2 * 40 * 50 and eP == [0.0, 1.0] and abs(eA - 30.0) <= TOL_DEG
    z = torch.zeros((0, 3, 40, 50), device="cuda")
    assert ctx.accuracy(z, z, None, (1.0,)) == (0.0, [0.0], 0)
    mz = torch.zeros((2, 40, 50), dtype=torch.uint8, device="cuda")
    assert ctx.accuracy(est, gt, mz, (1.0,)) == (0.0, [0.0], 0)
    eA0, eP0, m0 = ctx.accuracy(est, gt, None, ())  # no thresholds
    assert eP0 == [] and m0 == m and abs(eA0 - eA) <= 1e-12


def test_accuracy_calls_on_two_streams():
    """Calls on two streams share the context's scratch table; the second
    waits for the first, so both results are right."""
    shape = (4, 120, 160)
    rng = np.random.default_rng(24)
    t1 = rng.uniform(0.0, 40.0, size=shape)
    t2 = rng.uniform(60.0, 120.0, size=shape)
    e1, g1 = _rotated(25, shape, t1)
    e2, g2 = _rotated(26, shape, t2)
    ctx = sne.Context(0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    r1 = torch.empty(3, dtype=torch.float64, device="cuda")
    r2 = torch.empty(3, dtype=torch.float64, device="cuda")
    ph = (ctypes.c_float * 1)(20.0)
    L = sne.lib()
    for e, g, r, s in ((e1, g1, r1, s1), (e2, g2, r2, s2)):
        assert L.sne_accuracy(ctx.handle, e.data_ptr(), 0, g.data_ptr(), None, shape[0],
                              shape[1] * shape[2], ph, 1, r.data_ptr(), s.cuda_stream) == 0
    torch.cuda.synchronize()
    assert abs(r1[0].item() - t1.mean()) <= TOL_DEG and abs(r2[0].item() - t2.mean()) <= TOL_DEG
    assert int(r1[1].item()) == t1.size and r2[2].item() == 0.0
