"""GPU parity of the operators against the CPU float64 oracle (through the C ABI).

Tolerances: float32 path relative L2 <= 1e-5 (projector, backprojector, WMG
apply), float64 path <= 1e-12; packet diagonal elementwise relative 1e-5 / 1e-12
(every coefficient against its own oracle value; a zero oracle value must be an
exact zero, since the apply takes 1/0 := 0).  The level counts run from 1 to 6
(packet tiles of 1 to 32 pixels), so every instantiation of the packet-diagonal
kernel, the fused backprojector apply (tiles up to 16) and the separate apply
(32) is compared with the oracle.
"""
import numpy as np
import pytest

from gpu_common import check_diag_elementwise, oracle_W, oracle_d, print_case, rel, to_gpu, to_np
from oracle import wmg
from oracle.geometry import Geometry as OG
from oracle.projector import pixel_column, ray_rows

torch = pytest.importorskip("torch")
reco = pytest.importorskip("paper_1310_0956_amd")

pytestmark = pytest.mark.gpu

# (n, m, nb, levels, f64): ragged sizes, the paper's 40x40 geometry, the 64^2 FP64
# workload, axis-only and 45-degree angle sets, a single pixel-pair image.
CASES = [
    (24, 18, 35, 3, False),
    (40, 100, 40, 2, False),
    (64, 90, 64, 2, True),
    (64, 90, 64, 2, False),
    (48, 2, 70, 2, False),
    (32, 4, 45, 4, True),
    (2, 3, 3, 1, False),
    (16, 1, 1, 2, True),
    (128, 37, 182, 3, False),
    # five and six levels: 16x16 and 32x32 packet tiles
    (64, 90, 91, 5, False),
    (64, 90, 91, 5, True),
    (128, 37, 182, 5, False),
    (128, 37, 182, 5, True),
    (64, 45, 91, 6, False),
    (64, 45, 91, 6, True),
    # odd tile counts per side (the centre tile is its own mirror), even and odd m
    (48, 30, 70, 5, False),
    (48, 30, 70, 5, True),
    (40, 21, 57, 4, False),
    (40, 21, 57, 4, True),
    (24, 12, 35, 4, True),
    # small images whose 32-bin forward blocks span the whole shadow: the first
    # and last ray of a block miss the image on either side while the rays
    # between them cross it (axis-parallel and sloped angles)
    (24, 2, 35, 3, True),
    (16, 2, 23, 3, False),
    (14, 6, 33, 2, False),
    (14, 6, 33, 2, True),
    # few angles on a large image: a group of consecutive angles spans up to
    # 165 degrees, so band windows reach 238 columns and the forward projector
    # reads those bands straight from memory
    (256, 12, 363, 2, False),
    (256, 12, 363, 2, True),
]
TOL = {False: 1e-5, True: 1e-12}


def _img(n, seed):
    rng = np.random.default_rng(seed)
    return rng.random((n, n)) + (rng.random((n, n)) > 0.8)


@pytest.mark.parametrize("n,m,nb,lv,f64", CASES)
def test_project_backproject_wmg_parity(n, m, nb, lv, f64):
    print_case("operators", n, m, nb, lv, f64)
    dt = torch.float64 if f64 else torch.float32
    g = reco.Geometry(n, m, nb, lv, reco.F64 if f64 else reco.F32)
    W = oracle_W(n, m, nb)
    x = _img(n, 1)
    xs = to_gpu(x, dt)
    x_dev = to_np(xs)   # the exact values the GPU sees
    b = to_np(g.project(xs))
    assert rel(b, W @ x_dev.ravel()) <= TOL[f64]
    y = np.random.default_rng(2).standard_normal((m, nb))
    ys = to_gpu(y, dt)
    y_dev = to_np(ys)
    bt = to_np(g.backproject(ys))
    assert rel(bt, W.T @ y_dev.ravel()) <= TOL[f64]
    # adjoint identity with the GPU operators themselves, for a nonnegative y:
    # x and W are nonnegative, so <W x, y> sums nonnegative terms and its
    # relative error is that of the terms' rounding (with the random-sign y
    # above it cancels, up to 443 times on these geometries)
    ya = to_gpu(np.abs(y_dev), dt)
    ya_dev = to_np(ya)
    bta = to_np(g.backproject(ya))
    lhs = float(np.dot(b.ravel(), ya_dev.ravel()))
    rhs = float(np.dot(x_dev.ravel(), bta.ravel()))
    assert abs(lhs - rhs) <= (1e-12 if f64 else 2e-6) * abs(lhs)
    # packet diagonal and WMG apply
    L = lv - 1
    d_ref = oracle_d(n, m, nb, L)
    d = g.packet_diagonal()
    check_diag_elementwise(d, d_ref, TOL[f64])
    for lam in (0.0, 0.37):
        z = to_np(g.wmg_apply(xs, lam=lam))
        z_ref = wmg.apply_additive_diag(x_dev, d_ref + lam, L)
        print("wmg apply lam", lam, "rel err", rel(z, z_ref), flush=True)
        assert rel(z, z_ref) <= TOL[f64]


# Deep hierarchies (ell = 5, 6) through the float64 solver: 10 WMG-CGLS
# iterations, iterates and residual histories within 1e-8 of the oracle's.
@pytest.mark.parametrize("n,m,nb,lv", [(64, 90, 91, 5), (128, 37, 182, 5), (64, 45, 91, 6)])
def test_deep_wmg_cgls_f64(n, m, nb, lv):
    from oracle import solvers
    import inputs
    print_case("deep wmg-cgls f64", n, m, nb, lv)
    W = oracle_W(n, m, nb)
    b = W @ inputs.ellipse_phantom(n, 10, 5).ravel()
    L = lv - 1
    d_ref = oracle_d(n, m, nb, L)
    ref = solvers.pcgls(W, b, fixed_iters=10,
                        precond=lambda v: wmg.apply_additive_diag(v, d_ref, L))
    g = reco.Geometry(n, m, nb, lv, reco.F64)
    x, info = g.solve_cgls(to_gpu(b.reshape(m, nb), torch.float64), fixed_iters=10,
                           history=True)
    assert info["iters"] == 10 and info["status"] == "ok"
    print("deep wmg-cgls rel err", rel(to_np(x), ref.x), flush=True)
    assert rel(to_np(x), ref.x) <= 1e-8
    assert np.allclose(info["history"], ref.history, rtol=1e-8)


def test_project_ct512_full():
    n, m, nb, lv = 512, 360, 725, 3
    print_case("ct512 operators")
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    W = oracle_W(n, m, nb)
    import inputs
    x = inputs.ellipse_phantom(n, 20, 1000)
    xs = to_gpu(x, torch.float32)
    b = to_np(g.project(xs))
    assert rel(b, W @ x.ravel()) <= 1e-5
    y = np.random.default_rng(3).standard_normal((m, nb))
    ys = to_gpu(y, torch.float32)
    y_dev = to_np(ys)
    assert rel(to_np(g.backproject(ys)), W.T @ y_dev.ravel()) <= 1e-5
    assert g.count_nnz() == pytest.approx(W.nnz, rel=1e-4)
    d_ref = oracle_d(n, m, nb, lv - 1)
    check_diag_elementwise(g.packet_diagonal(), d_ref, 1e-5)
    z = to_np(g.wmg_apply(xs))
    assert rel(z, wmg.apply_additive_diag(x, d_ref, lv - 1)) <= 1e-5


def test_ct2048_sampled():
    """2048^2, 2048 angles, 2897 bins, 5 WMG levels at full size: sampled rays
    and pixels of W and W^T, and the packet diagonal and WMG apply on sampled
    16x16 packet tiles."""
    n, m, nb, lv = 2048, 2048, 2897, 5
    print_case("ct2048 sampled operators")
    og = OG(n, m, nb)
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    import inputs
    x = inputs.ellipse_phantom(n, 40, 2000)
    xs = to_gpu(x, torch.float32)
    b = to_np(g.project(xs)).reshape(m, nb)
    rng = np.random.default_rng(7)
    angles = sorted(set([0, 1, m // 4, m // 2, m // 2 + 1, 3 * m // 4, m - 1]
                        + list(rng.integers(0, m, 9))))
    for k in angles:
        bins = np.unique(np.concatenate([[0, nb // 2, nb - 1], rng.integers(0, nb, 24)]))
        ref = ray_rows(og, int(k), bins) @ x.ravel()
        got = b[k, bins]
        assert rel(got, ref) <= 1e-5, k
    y = rng.standard_normal((m, nb)).astype(np.float32)
    ys = to_gpu(y, torch.float32)
    bt = to_np(g.backproject(ys)).ravel()
    y64 = y.astype(np.float64).ravel()
    for pix in [0, n - 1, n * n - 1, (n // 2) * n + n // 2] + list(rng.integers(0, n * n, 4)):
        col = pixel_column(og, int(pix))
        ref = col @ y64
        # rounding bound: 1e-5 of the sum of |terms|
        assert abs(bt[pix] - ref) <= 1e-5 * (np.abs(col) @ np.abs(y64)), pix
    # packet diagonal and WMG apply on sampled 16x16 packet tiles (L = 4: each
    # coefficient is a Walsh pattern on one tile, so a tile's coefficients need
    # only the tile's 256 columns of W; a coefficient at local quadrant-layout
    # position (r, c) sits at (n/16 r + tile row, n/16 c + tile column) of the
    # whole image's quadrant layout)
    import scipy.sparse as sp
    d_gpu = g.packet_diagonal()
    s_img = rng.standard_normal((n, n)).astype(np.float32)
    z_gpu = to_np(g.wmg_apply(to_gpu(s_img, torch.float32))).reshape(n, n)
    T, S = 16, n // 16
    for ty, tx in [(0, 0), (57, 83)]:
        cols = []
        for iy in range(T):
            for ix in range(T):
                cols.append(sp.csr_matrix(pixel_column(og, (ty * T + iy) * n + tx * T + ix)).T)
        Wt = sp.hstack(cols).tocsr()                     # M x 256, local pixel order
        d_loc = wmg.packet_diagonal(Wt, T, 4)
        d_tile = d_gpu[ty::S, tx::S]                     # the tile's coefficients, local layout
        check_diag_elementwise(d_tile, d_loc, 1e-5)
        s_tile = s_img[ty * T:(ty + 1) * T, tx * T:(tx + 1) * T].astype(np.float64)
        z_ref = wmg.apply_additive_diag(s_tile, d_loc, 4)
        z_tile = z_gpu[ty * T:(ty + 1) * T, tx * T:(tx + 1) * T]
        print("ct2048 tile", ty, tx, "wmg apply rel err", rel(z_tile, z_ref), flush=True)
        assert rel(z_tile, z_ref) <= 1e-5
