"""GPU stage parity through the C ABI: canonical rays and the occupancy
march bit-exact, hash encoding and MLPs within tolerance of the FP64
oracle."""
import math

import numpy as np
import pytest

from mlp_bound import mlp16_bounds, mlp16_rgb_rms_bound
from gpu_common import F32, axis_camera, need_gpu, tiny_field
from oracle.encoding import encode, level_star, lod_weights
from oracle.march import dense_masked_march
from oracle.mlp import color_mlp, density_mlp
from oracle.rays import canonical_rays, cone_pitch
from oracle.sh import sh_basis
from paper_2311_02542_amd import capi, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    need_gpu()
    r = capi.Renderer(0)
    yield r
    r.close()


def _rays(R, cams, W, H):
    torch = R.torch
    n = len(cams) * W * H
    o = torch.empty((n, 3), device="cuda")
    d = torch.empty((n, 3), device="cuda")
    r = torch.empty(n, device="cuda")
    capi.vrn_rays(R.ctx, cams, W, H, o, d, r)
    torch.cuda.synchronize()
    return o.cpu().numpy(), d.cpu().numpy(), r.cpu().numpy()


@pytest.mark.parametrize("case", ["blobs64", "room256", "house_stereo", "axis"])
def test_rays_bit_exact(R, case):
    if case == "blobs64":
        cams, W, H = synth.cameras_blobs64(4), 64, 64
    elif case == "room256":
        cams, W, H = synth.cameras_room256(2, 96, 72), 96, 72
    elif case == "house_stereo":
        cams, W, H = synth.cameras_house_stereo([0, 150], 80, 80)[1], 80, 80
    else:
        cams = [axis_camera(np.eye(3), [0.1, 0.2, 0.3]),
                axis_camera(np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]]), [0.5, 0.5, 0.5])]
        W, H = 8, 8
    o, d, r = _rays(R, cams, W, H)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for c, cam in enumerate(cams):
        sl = slice(c * W * H, (c + 1) * W * H)
        oo, dd = canonical_rays(cam, ii.ravel(), jj.ravel())
        assert np.array_equal(d[sl].view(np.uint32), dd.view(np.uint32)), "direction bits differ"
        assert np.array_equal(o[sl], oo)
        rr = cone_pitch(cam, ii.ravel(), jj.ravel())
        np.testing.assert_allclose(r[sl], rr, rtol=2e-5)


def _march(R, field, cams, W, H, max_k):
    torch = R.torch
    fid = R.load(field)
    n = len(cams) * W * H
    kl = torch.zeros((n, max_k), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    capi.vrn_march(R.ctx, fid, cams, W, H, kl, max_k, cnt)
    torch.cuda.synchronize()
    R.unload(fid)
    return kl.cpu().numpy(), cnt.cpu().numpy()


def _check_march(R, field, cams, W, H):
    max_k = int(field["max_samples"])
    kl, cnt = _march(R, field, cams, W, H, max_k)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    total = 0
    for c, cam in enumerate(cams):
        o, d = canonical_rays(cam, ii.ravel(), jj.ravel())
        ks, counts = dense_masked_march(field, o, d)
        sl = slice(c * W * H, (c + 1) * W * H)
        assert np.array_equal(cnt[sl], counts), f"cam {c}: {np.sum(cnt[sl] != counts)} count mismatches"
        for p in np.nonzero(counts)[0]:
            assert np.array_equal(kl[sl][p, :counts[p]], ks[p, :counts[p]]), (c, p)
        total += counts.sum()
    return total


def test_march_bit_exact_blobs64(R):
    assert _check_march(R, synth.field_blobs64(), synth.cameras_blobs64(6), 64, 64) > 1000


def test_march_bit_exact_room256(R):
    f = synth.field_room256()
    assert _check_march(R, f, synth.cameras_room256(2, 72, 56), 72, 56) > 1000


@pytest.mark.parametrize("g", [1, 2, 3, 4, 8, 33])
def test_march_bit_exact_tiny_adversarial(R, g):
    rng = np.random.default_rng(100 + g)
    occ = rng.uniform(size=(g, g, g)) < 0.4
    occ[0, 0, 0] = True
    amin, ext = (-0.25, 0.5, 1.0), 1.5
    f = tiny_field(g, occ, amin, ext, cap=10000, seed=g)
    cell = ext / g
    cams = []
    perms = [np.eye(3), np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]]), np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]]),
             -np.eye(3) * np.array([1, -1, 1])]
    for k in range(8):   # origins on cell faces / edges / corners, inside and outside
        pos = np.array(amin) + cell * np.array([k % g + (k % 2) * 0.5, (k * 7) % (g + 1), (k * 3) % (g + 1)])
        if k % 3 == 0:
            pos = pos - 0.7 * ext
        cams.append(axis_camera(perms[k % 4], pos, fx=3.0 + k))
    assert _check_march(R, f, cams, 8, 8) >= 0


def test_march_empty_full_and_cap(R):
    g = 16
    f0 = tiny_field(g, np.zeros((g, g, g), bool))
    kl, cnt = _march(R, f0, synth.cameras_blobs64(2, 16, 16), 16, 16, 8)
    assert cnt.max() == 0
    f1 = tiny_field(g, np.ones((g, g, g), bool), cap=7)
    assert _check_march(R, f1, synth.cameras_blobs64(2, 16, 16), 16, 16) > 0
    kl, cnt = _march(R, f1, synth.cameras_blobs64(1, 16, 16), 16, 16, 7)
    assert cnt.max() == 7


def _sample_points(field, cams, W, H, n_max=20000):
    """Real sample positions (canonical FP32) with their t and cone pitch."""
    from oracle.march import canonical_positions
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    xs, ts, rs = [], [], []
    for cam in cams:
        o, d = canonical_rays(cam, ii.ravel(), jj.ravel())
        r = cone_pitch(cam, ii.ravel(), jj.ravel())
        ks, counts = dense_masked_march(field, o, d)
        for p in np.nonzero(counts)[0][::3]:
            k = ks[p, :min(counts[p], 4)]
            x, t = canonical_positions(o[p:p + 1], d[p:p + 1], k[None, :], field["dt"])
            xs.append(x[0]); ts.append(t[0]); rs.append(np.full(k.size, r[p]))
    x = np.concatenate(xs)[:n_max].astype(F32)
    return x, np.concatenate(ts)[:n_max].astype(F32), np.concatenate(rs)[:n_max].astype(F32)


@pytest.mark.parametrize("case", ["blobs64", "room256_lod", "house_levels_f16", "house_levels_f32"])
def test_encode_parity(R, case):
    torch = R.torch
    if case == "blobs64":
        f = synth.field_blobs64()
        x, t, r = _sample_points(f, synth.cameras_blobs64(4), 64, 64)
    elif case == "room256_lod":
        f = synth.field_room256()
        x, t, r = _sample_points(f, synth.cameras_room256(2, 64, 64), 64, 64)
    else:
        # the house field's level resolutions (up to N = 19912 over a 16 m cube) on a smaller table
        rng = np.random.default_rng(7)
        f = tiny_field(8, np.ones((8, 8, 8), bool), (0, 0, 0), 16.0, L=16, log2_T=16, lod=True,
                       bands=4, table_dtype=np.float16 if case.endswith("f16") else np.float32)
        f["level_res"] = synth.level_resolutions(16, 128.0, 1.4)
        f["base_res"], f["growth"] = 128.0, float(F32(1.4))
        x = rng.uniform(0, 16, (20000, 3)).astype(F32)
        t = rng.uniform(0.05, 12, 20000).astype(F32)
        r = np.full(20000, F32(1.0 / 859.24))
    fid = R.load(f)
    n = x.shape[0]
    L = int(f["n_levels"])
    dx, dt_, dr = (torch.from_numpy(a).cuda() for a in (x, t, r))
    feat = torch.full((n, 2 * L), float("nan"), device="cuda")
    capi.vrn_encode(R.ctx, fid, dx, dt_, dr, n, feat)
    torch.cuda.synchronize()
    R.unload(fid)
    g = feat.cpu().numpy()
    w = lod_weights(level_star(t.astype(np.float64), r.astype(np.float64), f), L) if f["lod_enable"] else None
    ref = encode(f, x, w)
    err = np.abs(g - ref)
    assert np.isfinite(g).all()
    assert err.max() <= 1e-6, f"max abs feature error {err.max():.3g}"


@pytest.mark.parametrize("compute", ["f32", "f32x", "f16", "bf16"])
@pytest.mark.parametrize("case", ["blobs64", "room256"])
def test_mlp_parity(R, case, compute):
    """FP32 (FP32 MFMA, or FP32 by split BF16 MFMA): sigma within 2e-6
    relative, RGB within 1e-6.  FP16 / BF16: per
    sample, sigma within the a-priori worst-case bound of the 16-bit
    arithmetic and RGB within six standard deviations of its rounding model
    (tests/mlp_bound.py, itself checked against a CPU emulation)."""
    torch = R.torch
    f = synth.field_blobs64() if case == "blobs64" else synth.field_room256()
    L = int(f["n_levels"])
    rng = np.random.default_rng(11)
    n = 4099  # ragged tail of a 16-sample tile
    feats = rng.uniform(-0.1, 0.1, (n, 2 * L)).astype(F32)
    d = rng.standard_normal((n, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(F32)
    fid = R.load(f)
    sig = torch.empty(n, device="cuda")
    rgb = torch.empty((n, 3), device="cuda")
    capi.vrn_mlp(R.ctx, fid, torch.from_numpy(feats).cuda(), torch.from_numpy(d).cuda(), n, compute, sig, rgb)
    torch.cuda.synchronize()
    R.unload(fid)
    s_ref, geo = density_mlp(feats.astype(np.float64), f["mlp"])
    sh = sh_basis(d.astype(np.float64), int(f["sh_bands"]))
    c_ref = color_mlp(geo, sh, f["mlp"])
    s_err = np.abs(sig.cpu().numpy() / s_ref - 1)
    c_err = np.abs(rgb.cpu().numpy() - c_ref)
    if compute in ("f32", "f32x"):
        tol_sig, tol_rgb = 2e-6, 1e-6
    else:
        tol_sig, _ = mlp16_bounds(feats, sh, f["mlp"], compute)
        tol_rgb = mlp16_rgb_rms_bound(feats, sh, f["mlp"], compute)
    print(f"{case} {compute}: sigma err / tol max {np.max(s_err / tol_sig):.3f}, "
          f"rgb err / tol max {np.max(c_err / tol_rgb):.3f}")
    assert (s_err <= tol_sig).all(), f"sigma rel err {np.max(s_err / tol_sig):.3g} x tolerance"
    assert (c_err <= tol_rgb).all(), f"rgb abs err {np.max(c_err / tol_rgb):.3g} x tolerance"


def test_march_bit_exact_clear_runs(R):
    """Long runs of clear coarse blocks (the block DDA path): occupied cells sit
    one cell across block boundaries and rays run along block faces, edges and
    through block corners, where a walk error would pass an occupied cell."""
    g = 128                                     # 4-cell coarse blocks, 32^3 of them
    occ = np.zeros((g, g, g), bool)
    rng = np.random.default_rng(7)
    for _ in range(60):                         # isolated cells just across block faces
        c = rng.integers(1, g // 4 - 1, size=3) * 4 + rng.choice([-1, 0], size=3)
        occ[c[2], c[1], c[0]] = True
    occ[:, :, 63] = True                        # a wall one cell before a block face (x = 64)
    occ[64, 20:100, 20:100] = True              # a slab on a block face (z = 64)
    f = tiny_field(g, occ, (0.0, 0.0, 0.0), 1.0, cap=4096, seed=3)
    cell = 1.0 / g
    cams = []
    perms = [np.eye(3), np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]]), np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]])]
    for k in range(9):
        # origins on block faces / edges / corners (multiples of 4 cells), some outside the grid
        pos = cell * 4 * np.array([1 + (5 * k) % 30, 2 + (7 * k) % 29, 3 + (11 * k) % 28], float)
        if k % 4 == 3:
            pos = pos - 0.6
        cams.append(axis_camera(perms[k % 3], pos, W=24, H=24, fx=6.0 + 2 * k, cx=12.0, cy=12.0))
    assert _check_march(R, f, cams, 24, 24) > 1000


def test_march_and_render_at_maximum_grid(R):
    """The largest occupancy grid the library accepts (G = 1024; 16-cell coarse
    blocks, 256^3 bricks) with 16 hashed levels: march bit-exact and the FP32
    image within 1e-5 PQ on sampled pixels."""
    from gpu_common import compare_render
    from oracle.render import render_fp64
    g = 1024
    occ = np.zeros((g, g, g), bool)
    occ[100:110, 200:900, 200:900] = True       # a thick floor-like slab (z)
    occ[300:700, 500:510, 300:700] = True       # a wall (y)
    occ[400:420, 400:420, 100:900] = True       # a beam (x)
    f = tiny_field(g, occ, (-2.0, -2.0, -2.0), 4.0, cap=2048, seed=11, L=16, log2_T=19, lod=True, b_sigma=3.0)
    f["dt"] = float(F32(4.0 * math.sqrt(3) / 2048))
    cams = [axis_camera(np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]]), [-1.5, 0.3, 0.1], W=16, H=16, fx=9.0,
                        cx=8.0, cy=8.0),
            axis_camera(np.eye(3), [0.1, -0.3, -1.9], W=16, H=16, fx=7.0, cx=8.0, cy=8.0)]
    assert _check_march(R, f, cams, 16, 16) > 500
    fid = R.load(f)
    rgba, ns = R.render(fid, cams, 16, 16, "f32")
    R.torch.cuda.synchronize()
    R.unload(fid)
    ref = render_fp64(f, cams, 16, 16)
    mx, _, _ = compare_render(rgba.cpu().numpy(), ns.cpu().numpy(), ref, 1e-5)
    assert mx <= 1e-5 and ref["n"].sum() > 100
