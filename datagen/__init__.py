"""Seeded synthetic workloads shared by the oracle tests and the HIP path.

This module only draws random numbers.  It holds none of the method's
arithmetic: no kernel-matrix entry, no softmax, no Hessian, no solve.  Latent
functions for the labels are drawn with random Fourier features (a spectral
sampler, Rahimi & Recht 2007) and class labels with the Gumbel-max trick, so
neither the exact kernel nor the likelihood is evaluated here.

Workloads (sizes follow the paper's experiments, see the paper's Section 5 and
its appendix on experimental details):

* ``config1``  N=512,  D=4,   C=3,  Matern-3/2 (l=1, os=1); X ~ N(0, I).
* ``config2``  N=20000, D=16, C=5,  Matern-5/2 (l=2, os=1); X ~ N(0, I).
* ``config3``  N=60000, D=784, C=10, RBF; image-shaped inputs in [0, 1] with
  ~80% exact zeros (a synthetic stand-in for the MNIST experiment).
* ``config4``  64 independent problems, N ~ U{1000..16000}, C ~ U{2..8}, D=8.
* ``config5``  fitted model N=100000, D=32, C=10, RBF; request stream.
* ``gmm``      the paper's 3-D Gaussian-mixture classification workload.
* ``poisson``  the paper's 1-D Poisson regression workload.

Every generator is a pure function of its seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

KERNEL_KINDS = ("rbf", "matern12", "matern32", "matern52")
# integer codes shared with the C ABI (igp_kernel_kind)
KERNEL_CODE = {"rbf": 0, "matern12": 1, "matern32": 2, "matern52": 3}
_MATERN_NU = {"matern12": 0.5, "matern32": 1.5, "matern52": 2.5}


@dataclasses.dataclass
class Workload:
    """One classification problem: inputs, labels and the fixed prior."""

    name: str
    X: np.ndarray            # (N, D) float64
    y: np.ndarray            # (N,) int32 in [0, C)
    C: int
    kernel: str
    lengthscale: float
    outputscale: float
    Xs: Optional[np.ndarray] = None   # test inputs (Ns, D)
    ys: Optional[np.ndarray] = None   # test labels
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.X.shape[0])

    @property
    def D(self) -> int:
        return int(self.X.shape[1])


def rff_frequencies(rng: np.random.Generator, kind: str, D: int, F: int) -> np.ndarray:
    """Frequencies from the kernel's spectral density (unit lengthscale).

    RBF: standard normal.  Matern-nu: multivariate Student-t with 2*nu degrees
    of freedom, i.e. z / sqrt(u / (2 nu)) with z ~ N(0, I), u ~ chi^2(2 nu).
    """
    z = rng.standard_normal((F, D))
    if kind == "rbf":
        return z
    nu = _MATERN_NU[kind]
    u = rng.chisquare(2.0 * nu, size=(F, 1))
    return z / np.sqrt(u / (2.0 * nu))


def rff_gp_draw(rng: np.random.Generator, X: np.ndarray, kind: str,
                lengthscale: float, outputscale: float, n_out: int,
                F: int = 2048, Xs: Optional[np.ndarray] = None):
    """Approximate draws of ``n_out`` independent zero-mean GPs at X (and Xs).

    f(x) = sqrt(2 os / F) * sum_k w_k cos(omega_k . x / l + b_k), w ~ N(0,1),
    b ~ U(0, 2 pi).  Returns arrays of shape (N, n_out) (and (Ns, n_out)).
    """
    D = X.shape[1]
    om = rff_frequencies(rng, kind, D, F) / lengthscale
    b = rng.uniform(0.0, 2.0 * math.pi, size=F)
    w = rng.standard_normal((F, n_out))
    scale = math.sqrt(2.0 * outputscale / F)

    def feat(A):
        out = np.empty((A.shape[0], n_out))
        for i0 in range(0, A.shape[0], 8192):
            blk = A[i0:i0 + 8192]
            out[i0:i0 + 8192] = (np.cos(blk @ om.T + b) * scale) @ w
        return out

    fx = feat(X)
    return (fx, feat(Xs)) if Xs is not None else fx


def gumbel_max_labels(rng: np.random.Generator, logits: np.ndarray) -> np.ndarray:
    """Categorical draws with P(y=c) proportional to exp(logit_c) (Gumbel-max)."""
    g = -np.log(-np.log(rng.uniform(np.finfo(float).tiny, 1.0, size=logits.shape)))
    return np.argmax(logits + g, axis=1).astype(np.int32)


def gp_classification(seed: int, N: int, D: int, C: int, kernel: str,
                      lengthscale: float, outputscale: float, Ns: int = 0,
                      F: int = 2048, name: str = "gpc") -> Workload:
    """X ~ N(0, I_D); labels from the softmax of a (RFF) GP draw per class."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, D))
    Xs = rng.standard_normal((Ns, D)) if Ns > 0 else None
    if Xs is not None:
        fx, fs = rff_gp_draw(rng, X, kernel, lengthscale, outputscale, C, F, Xs)
    else:
        fx, fs = rff_gp_draw(rng, X, kernel, lengthscale, outputscale, C, F), None
    y = gumbel_max_labels(rng, fx)
    ys = gumbel_max_labels(rng, fs) if fs is not None else None
    return Workload(name, X, y, C, kernel, lengthscale, outputscale, Xs, ys,
                    meta={"seed": seed, "rff_features": F})


def config1(seed: int = 0) -> Workload:
    """N=512, D=4, C=3, Matern-3/2 (l=1, os=1); 256 test points."""
    return gp_classification(seed, 512, 4, 3, "matern32", 1.0, 1.0, Ns=256, name="config1")


def config2(seed: int = 1, N: int = 20000, Ns: int = 2000) -> Workload:
    """N=20000, D=16, C=5, Matern-5/2 (l=2, os=1); 2000 test points."""
    return gp_classification(seed, N, 16, 5, "matern52", 2.0, 1.0, Ns=Ns, name="config2")


def image_like(seed: int = 2, N: int = 60000, Ns: int = 10000, C: int = 10,
               side: int = 28, support_frac: float = 0.2, noise: float = 0.1,
               blur_sigma: float = 2.0) -> Workload:
    """Image-shaped inputs in [0, 1], ~80% exact zeros (config 3).

    Per class: a support mask covering the top ``support_frac`` of a
    Gaussian-blurred N(0,1) field, intensities U(0.5, 1) on the support.
    Samples: clip(mean_c + noise * eps, 0, 1) on the support, exactly 0 off
    it, quantised to k/255.  Balanced classes.  The lengthscale is the median
    pairwise distance of a 2000-point subsample (median heuristic).
    """
    rng = np.random.default_rng(seed)
    D = side * side
    rad = int(math.ceil(3 * blur_sigma))
    t = np.arange(-rad, rad + 1)
    g1 = np.exp(-0.5 * (t / blur_sigma) ** 2)
    g1 /= g1.sum()
    means = np.zeros((C, D))
    masks = np.zeros((C, D), dtype=bool)
    for c in range(C):
        field = rng.standard_normal((side + 2 * rad, side + 2 * rad))
        # separable blur (valid region)
        rows = np.apply_along_axis(lambda r: np.convolve(r, g1, mode="valid"), 1, field)
        blurred = np.apply_along_axis(lambda r: np.convolve(r, g1, mode="valid"), 0, rows)
        flat = blurred.reshape(-1)
        thr = np.quantile(flat, 1.0 - support_frac)
        m = flat >= thr
        masks[c] = m
        means[c, m] = rng.uniform(0.5, 1.0, size=int(m.sum()))

    def draw(n):
        lab = np.repeat(np.arange(C), int(math.ceil(n / C)))[:n]
        rng.shuffle(lab)
        Xo = np.empty((n, D), dtype=np.float32)
        for i0 in range(0, n, 8192):
            li = lab[i0:i0 + 8192]
            blk = means[li] + noise * rng.standard_normal((li.size, D))
            blk = np.clip(blk, 0.0, 1.0) * masks[li]
            Xo[i0:i0 + 8192] = np.round(blk * 255.0) / 255.0
        return Xo.astype(np.float64), lab.astype(np.int32)

    X, y = draw(N)
    Xs, ys = draw(Ns) if Ns > 0 else (None, None)
    sub = rng.choice(N, size=min(2000, N), replace=False)
    A = X[sub]
    sq = (A * A).sum(1)
    d2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * A @ A.T, 0.0)
    iu = np.triu_indices(A.shape[0], 1)
    ell = float(np.median(np.sqrt(d2[iu])))
    return Workload("config3", X, y, C, "rbf", ell, 1.0, Xs, ys,
                    meta={"seed": seed, "zero_frac": float((X == 0).mean())})


def config3(seed: int = 2, N: int = 60000, Ns: int = 10000) -> Workload:
    return image_like(seed, N, Ns)


def config4(seed: int = 3, n_problems: int = 64, n_lo: int = 1000,
            n_hi: int = 16000, c_lo: int = 2, c_hi: int = 8, D: int = 8, F: int = 512):
    """Many independent problems of uneven size (batched form); RFF draws with
    ``F`` features per problem."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(n_lo, n_hi + 1, size=n_problems)
    Cs = rng.integers(c_lo, c_hi + 1, size=n_problems)
    seeds = rng.integers(0, 2**31 - 1, size=n_problems)
    return [gp_classification(int(s), int(n), D, int(c), "matern32", 1.0, 1.0, F=F,
                              name=f"config4[{i}]")
            for i, (n, c, s) in enumerate(zip(Ns, Cs, seeds))]


def config5_model(seed: int = 4, N: int = 100000, D: int = 32, C: int = 10,
                  F: int = 4096) -> Workload:
    """Fitted-model data for the serving workload (RBF, median lengthscale)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, D))
    ell = math.sqrt(2.0 * D)  # median distance of two N(0, I_D) points ~ sqrt(2D)
    fx = rff_gp_draw(rng, X, "rbf", ell, 1.0, C, F)
    y = gumbel_max_labels(rng, fx)
    return Workload("config5", X, y, C, "rbf", ell, 1.0, meta={"seed": seed})


def config5_requests(seed: int = 5, n_requests: int = 256, rate_hz: float = 100.0,
                     fit_frac: float = 0.05, D: int = 32, max_pred: int = 4096,
                     fit_lo: int = 2000, fit_hi: int = 50000):
    """Poisson request stream: predictive queries (log-uniform 1..4096 points)
    mixed with new fits (N ~ U{2000..50000})."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    reqs = []
    for i in range(n_requests):
        if rng.uniform() < fit_frac:
            n = int(rng.integers(fit_lo, fit_hi + 1))
            reqs.append({"t": float(t[i]), "kind": "fit", "n": n,
                         "seed": int(rng.integers(0, 2**31 - 1))})
        else:
            n = int(math.ceil(math.exp(rng.uniform(0.0, math.log(max_pred)))))
            reqs.append({"t": float(t[i]), "kind": "predict",
                         "X": rng.standard_normal((n, D))})
    return reqs


def config5_fit(seed: int, N: int, D: int = 32, C: int = 10, F: int = 1024) -> Workload:
    """Training data of one fit request of the serving stream (same prior as
    the served model: RBF with lengthscale sqrt(2D), outputscale 1)."""
    return gp_classification(seed, N, D, C, "rbf", math.sqrt(2.0 * D), 1.0, F=F,
                             name=f"config5-fit[{N}]")


def gmm(seed: int = 6, per_class: int = 10000, per_class_test: int = 1000,
        C: int = 10, D: int = 3, mix_seed: int = 1234) -> Workload:
    """3-D Gaussian mixture (the paper's large-scale classification data).

    Class means ~ U[-1, 1]^3; covariance U diag(lam) U^T with U the
    eigenvectors of A A^T (A with U(0,1) entries) and lam ~ U(0.001, 0.1).
    The mixture is fixed by ``mix_seed``; ``seed`` draws the samples.
    Matern-3/2 prior with lengthscale 0.05 and outputscale 0.05.
    """
    mrng = np.random.default_rng(mix_seed)
    mus = mrng.uniform(-1.0, 1.0, size=(C, D))
    covs = []
    for _ in range(C):
        A = mrng.uniform(0.0, 1.0, size=(D, D))
        _, U = np.linalg.eigh(A @ A.T)
        lam = mrng.uniform(0.001, 0.1, size=D)
        covs.append((U * lam) @ U.T)
    rng = np.random.default_rng(seed)

    def draw(k):
        X = np.concatenate([rng.multivariate_normal(mus[c], covs[c], size=k) for c in range(C)])
        y = np.repeat(np.arange(C), k).astype(np.int32)
        p = rng.permutation(X.shape[0])
        return X[p], y[p]

    X, y = draw(per_class)
    Xs, ys = draw(per_class_test)
    return Workload("gmm", X, y, C, "matern32", 0.05, 0.05, Xs, ys, meta={"seed": seed})


def poisson(seed: int = 7, N: int = 100, draw_seed: int = 66):
    """1-D Poisson regression data: X linspace(0, 1), log rate from an RBF GP
    (l=0.1, os=5), counts ~ Poisson(exp f).  ``draw_seed`` fixes the latent
    log rate; ``seed`` re-draws the counts.  The default draw keeps the log
    rate in [-2.3, 2.6] (counts up to ~19): on draws with rates in the
    hundreds, full Newton steps from f_0 = 0 overshoot and diverge."""
    X = np.linspace(0.0, 1.0, N)[:, None]
    frng = np.random.default_rng(draw_seed)
    f = rff_gp_draw(frng, X, "rbf", 0.1, 5.0, 1, F=4096)[:, 0]
    rng = np.random.default_rng(seed)
    y = rng.poisson(np.exp(f)).astype(np.int32)
    return X, y, f
