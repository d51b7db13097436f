"""Helpers for GPU parity tests: oracle systems cached per geometry, tensor moves."""
import functools
import math

import numpy as np

import inputs
from oracle import wmg
from oracle.geometry import Geometry as OG
from oracle.projector import system_matrix


@functools.lru_cache(maxsize=6)
def oracle_W(n, m, nb):
    return system_matrix(OG(n, m, nb))


@functools.lru_cache(maxsize=6)
def oracle_d(n, m, nb, L):
    return wmg.packet_diagonal(oracle_W(n, m, nb), n, L)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def to_gpu(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).astype(
        np.float64 if dtype == torch.float64 else np.float32)).cuda()


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def phantom_and_data(n, m, nb, n_ellipses, seed, noise=0.0, dtype64=False):
    """Seeded phantom, oracle sinogram b = W x (+ Gaussian noise), rounded to the storage type."""
    x = inputs.ellipse_phantom(n, n_ellipses, seed)
    W = oracle_W(n, m, nb)
    b = W @ x.ravel()
    if noise:
        b = b + noise * np.abs(b).max() * inputs.standard_normal(b.size, seed + 500000)
    if not dtype64:
        b = b.astype(np.float32).astype(np.float64)
    return x, b


def f32_store(eps, seed):
    """Float32 storage model for the oracle's kept vectors: a relative Gaussian
    error of size eps (a measured operator error), then rounding to float32."""
    g = np.random.default_rng(seed)
    return lambda v: (v * (1.0 + eps * g.standard_normal(np.shape(v)))).astype(
        np.float32).astype(np.float64)


def f32_envelope(run, ref_x, eps, seeds=5):
    """Largest deviation of an oracle run from ref_x under the float32 storage
    model (run(store) returns the oracle's result with that store hook)."""
    return max(rel(run(f32_store(eps, 100 + s)).x, ref_x) for s in range(seeds))


def operator_eps(g, W, x, y):
    """Relative L2 error of a float32 GPU geometry's projector and backprojector
    against the oracle's W and W^T (on the values the GPU sees)."""
    import torch
    xs, ys = to_gpu(x, torch.float32), to_gpu(y, torch.float32)
    x_dev, y_dev = to_np(xs).ravel(), to_np(ys).ravel()
    e_fwd = rel(to_np(g.project(xs)), W @ x_dev)
    e_bwd = rel(to_np(g.backproject(ys)), W.T @ y_dev)
    return e_fwd, e_bwd


def check_diag_elementwise(d, d_ref, tol):
    """Every packet coefficient within tol of its own oracle value."""
    d = np.asarray(d, dtype=np.float64).ravel()
    d_ref = np.asarray(d_ref, dtype=np.float64).ravel()
    zero = d_ref == 0.0
    assert np.all(d[zero] == 0.0), "packet diagonal: nonzero where the oracle has an exact zero"
    e = np.abs(d[~zero] - d_ref[~zero]) / d_ref[~zero]
    print("packet diagonal: max elementwise rel err", float(e.max(initial=0.0)),
          "zeros", int(zero.sum()), flush=True)
    assert e.max(initial=0.0) <= tol


def print_case(*args):
    print("CASE", *args, flush=True)


SQRT2 = math.sqrt(2.0)
