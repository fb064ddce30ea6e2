"""Seeded synthetic inputs shaped like the paper's workloads.

This module is the only code that the product and the oracle both use.  It
draws random data and rounds it once to its storage precision; it holds none of
the method's arithmetic (no problem mapping, no partition, no solver step).

Recipes (all numpy PCG64 ``default_rng(data_seed)``):

* least squares  -- D N x n iid N(0,1); x_true iid N(0,1); y = D x_true + 0.01 N(0,1).
  Stands in for the linear-regression use of Sec.3.1 (the lambda = 0 case).
* LASSO          -- D iid N(0,1) with columns scaled to unit l2 norm; x_true has
  nnz entries of random sign and magnitude U(1,3); y = D x_true + 0.05 N(0,1);
  lambda = frac * lambda_max with lambda_max = |D'y|_inf / (N alpha).  Stands in
  for the sparse-solution regression of Table 1 / Table 2 (dense data).
* elastic-net batch -- instance sizes log-uniform, Gaussian D, 10% of x_true
  non-zero, a 16-point log lambda grid per instance (Sec.3.1 cross-validation grids).
* SVM            -- two Gaussian classes with means +-0.5 * 1 and identity covariance,
  5% of labels flipped (stands in for the LIBSVM sets of Table 8, linear kernel).

Storage: data are generated in float64 and rounded once (round to nearest even)
to their storage type ("f64", "f32" or "bf16").  Both sides receive the rounded
values; for "bf16" the values are held in float32 arrays whose entries are
exactly representable in bfloat16.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def round_bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even); returns float32."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    bias = np.uint64(0x7FFF) + ((bits >> np.uint64(16)) & np.uint64(1))
    r = ((bits + bias) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).reshape(np.shape(a))


def to_storage(a, storage: str) -> np.ndarray:
    if storage == "f64":
        return np.asarray(a, dtype=np.float64)
    if storage == "f32":
        return np.asarray(a, dtype=np.float32)
    if storage == "bf16":
        return round_bf16(np.asarray(a, dtype=np.float32))
    raise ValueError(storage)


@dataclass
class RegressionWorkload:
    """Elastic-net family instance: min 1/(2N)|y - D x|^2 + lam*(alpha|x|_1 + (1-alpha)/2|x|^2)."""
    name: str
    D: np.ndarray          # N x n, Fortran order, values exact in `storage`
    y: np.ndarray          # N, float64
    lam: float
    alpha: float
    block_size: int
    beta0: float
    storage: str
    seed: int = 0          # partition seed
    x_true: np.ndarray | None = None

    @property
    def N(self):
        return self.D.shape[0]

    @property
    def n(self):
        return self.D.shape[1]


@dataclass
class SVMWorkload:
    """C-SVC dual instance (linear kernel): samples X (n x r) with labels y in {-1,+1}."""
    name: str
    X: np.ndarray          # n x r, C order (row i = sample i), values exact in `storage`
    labels: np.ndarray     # n, float64 in {-1, +1}
    C: float
    block_size: int
    beta0: float
    storage: str
    seed: int = 0

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def r(self):
        return self.X.shape[1]


def least_squares(N=2000, n=200, noise=0.01, data_seed=0, block_size=20, beta0=1.0,
                  storage="f64", name="ols") -> RegressionWorkload:
    rng = np.random.default_rng(data_seed)
    D = rng.standard_normal((N, n))
    x_true = rng.standard_normal(n)
    Ds = to_storage(D, storage)
    y = Ds.astype(np.float64) @ x_true + noise * rng.standard_normal(N)
    return RegressionWorkload(name, np.asfortranarray(Ds), y, 0.0, 1.0, block_size, beta0,
                              storage, 0, x_true)


def lasso(N=20000, n=2000, nnz_frac=0.05, noise=0.05, lam_frac=0.1, alpha=1.0, data_seed=2,
          block_size=64, storage="f32", normalize=True, name="lasso",
          beta0=None) -> RegressionWorkload:
    rng = np.random.default_rng(data_seed)
    D = rng.standard_normal((N, n))
    if normalize:
        D /= np.linalg.norm(D, axis=0, keepdims=True)
    nnz = max(1, int(round(nnz_frac * n)))
    x_true = np.zeros(n)
    pos = rng.choice(n, size=nnz, replace=False)
    x_true[pos] = rng.choice([-1.0, 1.0], size=nnz) * rng.uniform(1.0, 3.0, size=nnz)
    Ds = to_storage(D, storage)
    Df = Ds.astype(np.float64)
    y = Df @ x_true + noise * rng.standard_normal(N)
    lam_max = np.max(np.abs(Df.T @ y)) / (N * alpha)
    lam = lam_frac * lam_max
    b0 = 0.1 * lam if beta0 is None else beta0   # gamma = 0.1 lambda for dense data (Sec.3.1)
    return RegressionWorkload(name, np.asfortranarray(Ds), y, lam, alpha, block_size, b0,
                              storage, 0, x_true)


def gaussian_en(N, n, nnz_frac=0.1, noise=0.05, lam_frac=0.1, alpha=0.5, data_seed=3,
                block_size=64, storage="bf16", name="en", beta0=None) -> RegressionWorkload:
    """Gaussian (unnormalised) design; x_true with nnz_frac non-zeros drawn N(0,1)."""
    rng = np.random.default_rng(data_seed)
    D = rng.standard_normal((N, n), dtype=np.float32)
    nnz = max(1, int(round(nnz_frac * n)))
    x_true = np.zeros(n)
    pos = rng.choice(n, size=nnz, replace=False)
    x_true[pos] = rng.standard_normal(nnz)
    Ds = to_storage(D, storage)
    Df = Ds.astype(np.float64)
    y = Df @ x_true + noise * rng.standard_normal(N)
    lam_max = np.max(np.abs(Df.T @ y)) / (N * alpha)
    lam = lam_frac * lam_max
    b0 = 0.1 * lam if beta0 is None else beta0
    return RegressionWorkload(name, np.asfortranarray(Ds), y, lam, alpha, block_size, b0,
                              storage, 0, x_true)


def lambda_grid(lam_max, points=16, ratio=0.01):
    """lambda_j = lam_max * ratio^(j/(points-1)), j = 0..points-1 (a log grid)."""
    j = np.arange(points)
    return lam_max * ratio ** (j / (points - 1))


def en_batch_sizes(count=256, data_seed=3, Nlo=1000, Nhi=20000, nlo=100, nhi=4000):
    """Log-uniform instance sizes (N_i, n_i) for the batched elastic-net paths."""
    rng = np.random.default_rng(data_seed)
    N = np.round(np.exp(rng.uniform(np.log(Nlo), np.log(Nhi), size=count))).astype(np.int64)
    n = np.round(np.exp(rng.uniform(np.log(nlo), np.log(nhi), size=count))).astype(np.int64)
    return N, n


def svm(n=20000, r=256, shift=0.5, flip=0.05, Cbox=1.0, data_seed=4, block_size=128,
        storage="f32", name="svm", beta0=None) -> SVMWorkload:
    rng = np.random.default_rng(data_seed)
    labels = rng.choice([-1.0, 1.0], size=n)
    X = shift * labels[:, None] * np.ones((1, r)) + rng.standard_normal((n, r))
    nflip = int(round(flip * n))
    idx = rng.choice(n, size=nflip, replace=False)
    labels = labels.copy()
    labels[idx] = -labels[idx]
    Xs = to_storage(X, storage)
    p = -(-n // block_size)
    b0 = 0.1 * p if beta0 is None else beta0       # beta = 0.1 p (Sec.3.2)
    return SVMWorkload(name, np.ascontiguousarray(Xs), labels, float(Cbox), block_size, b0,
                       storage, 0)


# The five benchmark workloads ------------------------------------------------

def ols_2000x200():
    """Least squares, D 2000x200 FP64, p = 10 blocks of 20, beta = 1, 300 iterations, seed 0."""
    return least_squares(2000, 200, 0.01, 0, 20, 1.0, "f64", name="ols_2000x200")


def lasso_20000x2000(storage="f32"):
    """LASSO, D 20000x2000 unit-norm columns (FP32), 5% non-zeros, lambda = 0.1 lambda_max, s = 64."""
    return lasso(20000, 2000, 0.05, 0.05, 0.1, 1.0, 2, 64, storage, name="lasso_20000x2000")


def svm_20000x256():
    """SVM dual, 20000 samples x 256 features (FP32), C = 1, s = 128, beta = 0.1 p."""
    return svm(20000, 256, 0.5, 0.05, 1.0, 4, 128, "f32", name="svm_20000x256")


def lasso_10000x100000(storage="bf16"):
    """High-dimensional LASSO, D 10000x100000 (BF16), 1% non-zeros, lambda = 0.05 lambda_max, s = 128."""
    return gaussian_en(10000, 100000, 0.01, 0.05, 0.05, 1.0, 5, 128, storage,
                       name="lasso_10000x100000")


# Device-side generation for the large batched workload -------------------------

@dataclass
class DeviceRegression:
    """One instance generated on the GPU: F (n x N tensor, i.e. column-major N x n), y on the host."""
    F: object
    y: np.ndarray
    lam_max: float
    storage: str

    @property
    def N(self):
        return int(self.F.shape[1])

    @property
    def n(self):
        return int(self.F.shape[0])

    def host_D(self):
        """The instance's data as a float64 N x n array (exact copy of the stored values)."""
        return np.asfortranarray(self.F.float().cpu().numpy().T.astype(np.float64))


def en_instance_device(N, n, seed, nnz_frac=0.1, noise=0.05, alpha=0.5, storage="bf16", device="cuda", align=64):
    """Gaussian design N x n drawn with torch's seeded generator on the device, rounded once to
    `storage` (round to nearest even); x_true has nnz_frac non-zeros drawn N(0,1); y = D x_true +
    noise N(0,1); lam_max = |D'y|_inf / (N alpha).  Same values on every run for a given seed.
    Each column starts at a multiple of `align` elements (F is an (n, ldF)-strided view)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    dt = {"bf16": torch.bfloat16, "f32": torch.float32, "f64": torch.float64}[storage]
    ld = -(-N // align) * align
    buf = torch.zeros((n, ld), device=device, dtype=dt)
    buf[:, :N] = torch.randn((n, N), generator=g, device=device, dtype=torch.float32).to(dt)
    F = buf[:, :N]
    rng = np.random.default_rng(seed)
    nnz = max(1, int(round(nnz_frac * n)))
    xt = np.zeros(n)
    xt[rng.choice(n, size=nnz, replace=False)] = rng.standard_normal(nnz)
    xd = torch.as_tensor(xt, device=device)
    y = (F.double().T @ xd).cpu().numpy() + noise * rng.standard_normal(N)
    yd = torch.as_tensor(y, device=device)
    lam_max = float(torch.max(torch.abs(F.double() @ yd)).item()) / (N * alpha)
    return DeviceRegression(F, y, lam_max, storage)


# Dense-form workloads ----------------------------------------------------------

def svm_rbf(n=20000, r=128, n_test=5000, shift=1.5, flip=0.05, Cbox=1.0, data_seed=6, storage="f64"):
    """Gaussian-kernel C-SVC data (Sec.3.2): two Gaussian classes with means +-shift/sqrt(r) * 1
    (centres 2 shift apart) and identity covariance, a fraction `flip` of the training labels flipped; a held-out test set
    drawn from the same classes without flips.  gamma = 1/r (the common default of kernel SVM
    packages).  Returns (X, labels, X_test, labels_test, C, gamma), X row-major n x r."""
    rng = np.random.default_rng(data_seed)

    def draw(m):
        y = rng.choice([-1.0, 1.0], size=m)
        X = (shift / np.sqrt(r)) * y[:, None] * np.ones((1, r)) + rng.standard_normal((m, r))
        return to_storage(X, storage), y

    X, y = draw(n)
    idx = rng.choice(n, size=int(round(flip * n)), replace=False)
    y = y.copy()
    y[idx] = -y[idx]
    Xt, yt = draw(n_test)
    return np.ascontiguousarray(X), y, np.ascontiguousarray(Xt), yt, float(Cbox), 1.0 / r


def dense_qp_device(n=8192, meq=8, data_seed=7, device="cuda"):
    """General QP of Eq.(1) in the dense form, generated on the device: Hd = G'G/m + 0.01 I with
    G (m = n/2 rows) iid N(0,1) (symmetrised exactly), c iid N(0,1), meq equality rows A iid N(0,1)
    and beq = A x0 with x0 ~ U(0.1, 0.9) (feasible inside the box [0, 1]).  Returns torch tensors
    (Hd n x n float64, c, A, beq)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(data_seed))
    m = n // 2
    G = torch.randn((m, n), generator=g, device=device, dtype=torch.float64)
    H = (G.T @ G) / m
    H = 0.5 * (H + H.T) + 0.01 * torch.eye(n, device=device, dtype=torch.float64)
    del G
    c = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    A = torch.randn((meq, n), generator=g, device=device, dtype=torch.float64)
    x0 = 0.1 + 0.8 * torch.rand(n, generator=g, device=device, dtype=torch.float64)
    beq = A @ x0
    return H.contiguous(), c, A.contiguous(), beq


# Sparse workloads ----------------------------------------------------------------

@dataclass
class SparseRegression:
    """Elastic-net instance with sparse data in compressed sparse columns (numpy)."""
    name: str
    N: int
    n: int
    colptr: np.ndarray     # int64, n + 1
    rowidx: np.ndarray     # int32, nnz (strictly increasing within a column)
    values: np.ndarray     # float64 values exact in `storage`
    y: np.ndarray
    lam: float
    alpha: float
    storage: str

    def dense(self) -> np.ndarray:
        """The same data as a dense N x n float64 array (Fortran order)."""
        D = np.zeros((self.N, self.n), order="F")
        for j in range(self.n):
            a, b = self.colptr[j], self.colptr[j + 1]
            D[self.rowidx[a:b], j] = self.values[a:b]
        return D


def sparse_regression(N=2000, n=600, density=0.02, nnz_frac=0.5, noise=0.05, lam_frac=0.1, alpha=0.5,
                      data_seed=8, storage="f64", name="sparse_en") -> SparseRegression:
    """Sparse elastic-net data (stands in for the high-sparsity regressions of Sec.3.1, Tables 3-7):
    every column holds round(density N) entries at distinct uniformly drawn rows with N(0,1) values;
    x_true has a fraction nnz_frac of non-zeros N(0,1); y = D x_true + noise N(0,1);
    lambda = lam_frac lambda_max, lambda_max = |D'y|_inf / (N alpha)."""
    rng = np.random.default_rng(data_seed)
    k = max(1, int(round(density * N)))
    rows = np.stack([np.sort(rng.choice(N, size=k, replace=False)) for _ in range(n)]).astype(np.int32)
    vals = to_storage(rng.standard_normal((n, k)), storage).astype(np.float64)
    colptr = (np.arange(n + 1, dtype=np.int64) * k)
    rowidx = rows.reshape(-1)
    values = vals.reshape(-1)
    x_true = np.zeros(n)
    nz = rng.choice(n, size=max(1, int(round(nnz_frac * n))), replace=False)
    x_true[nz] = rng.standard_normal(nz.size)
    y = np.zeros(N)
    np.add.at(y, rowidx, values * np.repeat(x_true, k))
    y += noise * rng.standard_normal(N)
    Dty = np.zeros(n)
    for j in range(n):
        Dty[j] = values[j * k:(j + 1) * k] @ y[rowidx[j * k:(j + 1) * k]]
    lam = lam_frac * np.max(np.abs(Dty)) / (N * alpha)
    return SparseRegression(name, N, n, colptr, rowidx, values, y, float(lam), float(alpha), storage)


def sparse_regression_device(N, n, density, nnz_frac=0.5, noise=0.05, lam_frac=0.1, alpha=0.5, data_seed=9,
                             device="cuda"):
    """Large sparse elastic-net data generated on the device (torch's seeded generator): every column
    holds k = round(density N) entries at distinct rows -- the sorted draws of k integers from
    [0, N - k] plus 0, 1, ..., k - 1 -- with N(0,1) FP32 values; x_true with a fraction nnz_frac of
    N(0,1) non-zeros; y = D x_true + noise N(0,1); lambda = lam_frac lambda_max.
    Returns (colptr, rowidx, values, y, lam) as device tensors / floats."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(data_seed))
    k = max(1, int(round(density * N)))
    draws = torch.randint(0, N - k + 1, (n, k), generator=g, device=device, dtype=torch.int64)
    rows = torch.sort(draws, dim=1).values + torch.arange(k, device=device, dtype=torch.int64)[None, :]
    rowidx = rows.reshape(-1).to(torch.int32).contiguous()
    del draws, rows
    values = torch.randn(n * k, generator=g, device=device, dtype=torch.float32)
    colptr = torch.arange(n + 1, device=device, dtype=torch.int64) * k
    xt = torch.zeros(n, device=device, dtype=torch.float64)
    nz = torch.randperm(n, generator=g, device=device)[:max(1, int(round(nnz_frac * n)))]
    xt[nz] = torch.randn(nz.numel(), generator=g, device=device, dtype=torch.float64)
    y = torch.zeros(N, device=device, dtype=torch.float64)
    det = torch.are_deterministic_algorithms_enabled()
    torch.use_deterministic_algorithms(True)   # a fixed summation order, so y is the same on every run
    try:
        y.index_put_((rowidx.to(torch.int64),), values.double() * xt.repeat_interleave(k), accumulate=True)
    finally:
        torch.use_deterministic_algorithms(det)
    y += noise * torch.randn(N, generator=g, device=device, dtype=torch.float64)
    Dty = (values.double() * y[rowidx.to(torch.int64)]).reshape(n, k).sum(dim=1)
    lam = lam_frac * float(Dty.abs().max().item()) / (N * alpha)
    return colptr, rowidx, values, y, lam
