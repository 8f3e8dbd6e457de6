"""Per-element comparison of GPU gradients with the oracle's (Sec. 3.5).

Two levels, each with its own tolerance per element:

* 2D gradients (per Gaussian: mean x/y, conic a/b/c, opacity, colour), the
  sums over every pixel that blends the Gaussian, added in an order that
  atomics make arbitrary.  The float64 oracle gives each sum and a bound B on
  the magnitudes its terms are built from; a float32 evaluation in any order
  is within (n + m) * 2^-24 * B of the exact sum (first-order running-error
  analysis, Higham, Accuracy and Stability of Numerical Algorithms, ch. 3),
  with n the Gaussian's number of blends and m the operations of a term plus
  the blends of the pixel whose forward colour enters the term.
* Parameter gradients, the chain rule from those 2D gradients through EWA,
  Sigma, the quaternion and SH.  Reference: the float64 chain applied to the
  GPU's own 2D gradients, so only the chain's float32 rounding is left.  Its
  size per element is estimated by Monte-Carlo arithmetic (Parker, 1997):
  float32 evaluations of the same chain with inputs moved by one ulp; the
  tolerance is a multiple of their spread.  Sixteen such evaluations: a
  chain element near a branch of the chain (a clamp) spreads in two modes,
  which four evaluations can miss (a simulated float32 evaluation then
  exceeded 9x the tolerance; with sixteen, the worst of six was 0.4x).
"""
import numpy as np

import oracle

U = 2.0 ** -24
PARAMS = ("means", "scales", "rots", "opacities", "sh")


def check_grad2d(g2_gpu, g2_ref, bound, nterms, count_max, ops=64):
    tol = (nterms[:, None].astype(np.float64) + count_max + ops) * U * bound
    err = np.abs(g2_gpu.astype(np.float64) - g2_ref)
    bad = err > tol
    worst = float((err / np.maximum(tol, 1e-300)).max())
    assert not bad.any(), ("2D gradients", int(bad.sum()), worst, np.argwhere(bad)[:5].tolist())
    return worst


def _ulp_jitter(a, rng):
    a = np.asarray(a, np.float32)
    d = rng.integers(-1, 2, a.shape)
    out = np.where(d > 0, np.nextafter(a, np.float32(np.inf)), np.where(d < 0, np.nextafter(a, np.float32(-np.inf)), a))
    return out.astype(np.float32)


def chain_tolerance(scene, cam, g2, runs=16, seed=0):
    """Per-element spread of float32 chain-rule evaluations under one-ulp
    perturbations of the scene and the 2D gradients."""
    import copy
    ref = oracle.chain(scene, cam, g2)
    rng = np.random.default_rng(seed)
    spread = {k: np.zeros_like(v) for k, v in ref.items()}
    for r in range(runs + 1):
        sc = copy.deepcopy(scene)
        g = np.asarray(g2, np.float64)
        if r > 0:
            for name in ("means", "scales", "rots", "opacities", "sh"):
                setattr(sc, name, _ulp_jitter(getattr(sc, name), rng))
            g = _ulp_jitter(g.astype(np.float32), rng).astype(np.float64)
        g32 = oracle.chain(sc, cam, g, precision="f32")
        for k in spread:
            spread[k] = np.maximum(spread[k], np.abs(g32[k] - ref[k]))
    return ref, spread


def check_params(grads_gpu, scene, cam, g2_gpu, kappa=8.0, floor=1e-9):
    ref, spread = chain_tolerance(scene, cam, np.asarray(g2_gpu, np.float64))
    worst = {}
    for k in PARAMS:
        a = np.asarray(grads_gpu[k], np.float64)
        tol = kappa * spread[k] + floor * (np.abs(ref[k]).max() + 1e-300)
        err = np.abs(a - ref[k])
        bad = err > tol
        worst[k] = float((err / np.maximum(tol, 1e-300)).max())
        assert not bad.any(), (k, int(bad.sum()), worst[k], np.argwhere(bad)[:5].tolist())
    return worst


def grad2d_tolerance(bound, nterms, count_max, ops=64):
    return (nterms[:, None].astype(np.float64) + count_max + ops) * U * bound


def propagated_tolerance(scene, cam, tol2d):
    """Largest change of each parameter gradient that 2D gradients moved by
    at most tol2d (per component) can cause: the chain is linear in them."""
    out = None
    for c in range(9):
        m = np.zeros_like(tol2d)
        m[:, c] = tol2d[:, c]
        g = oracle.chain(scene, cam, m)
        if out is None:
            out = {k: np.abs(v) for k, v in g.items()}
        else:
            for k in out:
                out[k] += np.abs(g[k])
    return out
