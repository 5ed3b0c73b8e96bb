"""Differentiation form: the adjoint backward of the transform.

* adjoint dot-product identity <F x, y> = <x, F^H y> on the GPU path;
* torch.autograd.gradcheck in complex128 at small n (FP64 finite differences
  against the hand-written backward);
* loss L = sum w |F x|^2: GPU gradient against the FP64 oracle gradient
  2 F^H (w * F x) and against exact central differences at sampled
  coordinates (evaluated in FP64 on the CPU from the rank-one form, since the
  loss is quadratic the central difference has no truncation error).
"""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import announce, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def test_adjoint_dot_product(torch):
    import paper_0811_2535_amd as lf
    for t, dt, tol in ((10, np.complex128, 1e-12), (16, np.complex64, 2e-6)):
        n = 1 << t
        x = to_dev(datagen.signals(n, 1, dt, "normal", 21)[0])
        y = to_dev(datagen.signals(n, 1, dt, "normal", 22)[0])
        announce("adjoint dot n=2^%d" % t)
        Fx = lf.fft(x, -1)
        FHy = lf.fft(y, 1)
        lhs = torch.vdot(Fx.to(torch.complex128), y.to(torch.complex128))
        rhs = torch.vdot(x.to(torch.complex128), FHy.to(torch.complex128))
        assert abs(complex(lhs - rhs)) <= tol * abs(complex(lhs)), (t, complex(lhs), complex(rhs))


def test_gradcheck_c128(torch):
    import paper_0811_2535_amd as lf
    for t in (3, 6):
        n = 1 << t
        x = to_dev(datagen.signals(n, 2, np.complex128, "normal", 30 + t)).requires_grad_()
        announce("gradcheck n=2^%d" % t)
        for sign in (-1, 1):
            assert torch.autograd.gradcheck(lambda v: lf.LiftFFT.apply(v, sign), (x,),
                                            eps=1e-6, atol=1e-8)


@pytest.mark.parametrize("t,batch,dt,tol", [(12, 2, np.complex128, 1e-12),
                                            (22, 8, np.complex64, 1e-6),
                                            (24, 1, np.complex64, 1e-6)])
def test_weighted_power_loss_gradient(torch, t, batch, dt, tol):
    """Config 5 at n = 2^22, batch 8 (and a small c128 case); at 2^24 the
    transform and its adjoint run through the three-level lift."""
    import paper_0811_2535_amd as lf
    n = 1 << t
    x_np = datagen.signals(n, batch, dt, "normal", 5)
    w_np = datagen.real_weights(n, batch, 5)
    x = to_dev(x_np).requires_grad_()
    rdt = torch.float32 if dt == np.complex64 else torch.float64
    w = to_dev(w_np).to(rdt)
    announce("loss gradient n=2^%d batch=%d %s" % (t, batch, np.dtype(dt).name))
    y = lf.LiftFFT.apply(x, -1)
    loss = (w * (y.real ** 2 + y.imag ** 2)).sum()
    loss.backward()
    torch.cuda.synchronize()
    if t >= 24:
        assert lf.cached_plan(n, batch, x.dtype, x.device).info()["levels"] == 3
    g = to_np(x.grad)
    xr = x_np.astype(np.complex128)
    Fx = oracle.fft_batch(xr, -1)
    ref = 2.0 * oracle.fft_batch(w_np * Fx, 1)
    for b in range(batch):
        e = oracle.rel_l2(g[b], ref[b])
        assert e <= tol, (b, e)
    # Central differences at 64 seeded coordinates, in FP64 on the CPU.  With
    # y = F x and c_k = exp(-2 pi i j k / n) (column j of F),
    # L(x + h d e_j) = sum_k w_k |y_k + h d c_k|^2; the central difference
    # (L(+h) - L(-h)) / 2h is summed term by term, so no 1e13-sized totals
    # cancel, and it is exact for this quadratic loss up to rounding.
    h = 1e-3
    k = np.arange(n)
    idx = datagen.sample_indices(batch * n, 64 if t < 24 else 16, seed=55)
    for flat in idx:
        b, j = divmod(int(flat), n)
        c = np.exp(-2j * np.pi * ((j * k) % n) / n)
        yb, wb = Fx[b], w_np[b]
        def dL(d):
            up, dn = yb + h * d * c, yb - h * d * c
            return float(np.sum(wb * ((up.real ** 2 + up.imag ** 2) - (dn.real ** 2 + dn.imag ** 2)))) / (2 * h)
        fd = dL(1.0) + 1j * dL(1j)
        rms = float(np.sqrt(np.mean(np.abs(ref[b]) ** 2)))
        assert abs(g[b, j] - fd) <= 10 * tol * rms + 1e-9 * abs(fd), (b, j, g[b, j], fd, rms)
        assert abs(ref[b, j] - fd) <= 1e-9 * rms, (b, j, ref[b, j], fd)
