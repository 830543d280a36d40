"""Pins of the FP64 reference ray caster against closed forms, invariants and
library routines — never against itself.

Each test names what it pins.  Conventions the paper leaves open (camera
basis, pixel order, lattice) are restated where a test needs them; the
quantity checked is a closed form or an invariant of the method:

* axis-aligned orthographic MIP with nearest sampling is the brute-force max
  over each voxel column (bit-exact);
* a constant cube composites to alpha = 1 - exp(-kappa L), colour = rgb alpha,
  for every ray and camera (the chord L from an independent face-clipping
  computation), and early termination stops after a closed-form sample count;
* trilinear interpolation reproduces multilinear fields exactly;
* a zero-extinction transfer function, or a clip above the data, gives a
  zero image;
* a single bright voxel lights exactly the pixels its projection covers, at
  the pinhole projection of its centre (an inverse of ray generation);
* front-to-back order of two slabs gives C = c1 A1 + (1 - A1) c2 A2;
* the discrete compositing converges at second order to the continuous
  emission-absorption integral evaluated by adaptive quadrature;
* mirroring cube and camera mirrors the image; early termination changes
  the image by at most (1 - a_ert) max rgb;
* 16-bit storage decoding and round-to-nearest-even encoding equal numpy's
  and torch's.
"""
import math

import numpy as np
import pytest

import oracle
import synth

INF = math.inf


def ramp64(n=256, kmax=1.0):
    s = np.arange(n, dtype=np.float64) / (n - 1)
    return np.stack([s, 0.5 * s, 1.0 - s, kmax * s], axis=1)


def face_clip_chord(o, d, N, ortho):
    """Entry/exit parameters of the line o + t d through [-1/2, N-1/2]^3, found by
    intersecting the six face planes and keeping hits inside each face."""
    lo = -0.5
    hi = [N[0] - 0.5, N[1] - 0.5, N[2] - 0.5]
    ts = []
    for a in range(3):
        if d[a] == 0.0:
            continue
        for plane in (lo, hi[a]):
            t = (plane - o[a]) / d[a]
            p = o + t * d
            ok = True
            for b in range(3):
                if b != a and not (lo - 1e-9 <= p[b] <= hi[b] + 1e-9):
                    ok = False
            if ok:
                ts.append(t)
    if len(ts) < 2:
        return None
    t0, t1 = min(ts), max(ts)
    if not ortho:
        t0 = max(t0, 0.0)
    if t1 - t0 <= 1e-9:
        return None
    return t0, t1


def window_positions(cam, W, H):
    """Pixel-centre offsets along the camera right/up axes for an orthographic window."""
    sx = ((np.arange(W) + 0.5) / W - 0.5) * cam.ortho_w
    sy = (0.5 - (np.arange(H) + 0.5) / H) * cam.ortho_h
    return sx, sy


def basis(cam):
    f = np.subtract(cam.target, cam.eye).astype(np.float64)
    f /= np.linalg.norm(f)
    r = np.cross(f, cam.up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return f, r, u


@pytest.fixture(scope="module")
def tiny_cube():
    return synth.cube(synth.tiny().cube)


# ---------------------------------------------------------------------------
# P1: axis-aligned orthographic MIP with nearest sampling == column max
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("axis", ["z", "x", "y"])
@pytest.mark.parametrize("clip", [-INF, 3.0])
def test_p1_axis_mip_nearest_equals_column_max(tiny_cube, axis, clip):
    vol = tiny_cube
    nz, ny, nx = vol.shape
    W, H = 256, 256
    cam = synth.axis_camera(nx, ny, nz, axis, W, H)
    res = oracle.render(vol, mode=oracle.MIP, interp=oracle.NEAREST, camera=cam, width=W,
                        height=H, clip=clip, step=0.5)
    img = res["image"]
    f, r, u = basis(cam)
    sx, sy = window_positions(cam, W, H)
    c = np.asarray(cam.target)
    # world position of each pixel centre on the plane through the target
    P = c[None, None, :] + sx[None, :, None] * r[None, None, :] + sy[:, None, None] * u[None, None, :]
    ax = int(np.argmax(np.abs(f)))
    others = [a for a in range(3) if a != ax]
    N = (nx, ny, nz)
    colmax = vol.max(axis=2 - ax)  # collapse the viewing axis of [z][y][x]
    expected = np.full((H, W), -INF)
    for j in range(H):
        for i in range(W):
            idx = [0, 0, 0]
            ok = True
            for a in others:
                if not (-0.5 <= P[j, i, a] < N[a] - 0.5):
                    ok = False
                    break
                idx[a] = int(math.floor(P[j, i, a] + 0.5))
            if not ok:
                continue
            # colmax is indexed by the two remaining array axes in [z][y][x] order
            key = tuple(idx[a] for a in sorted(others, reverse=True))
            m = float(colmax[key])
            expected[j, i] = m if m >= clip else 0.0
    assert np.array_equal(img, expected)
    assert not np.any(res["flags"] & (oracle.FLAG_NEAREST_AMBIG | oracle.FLAG_GRAZE_AMBIG))
    hit = res["flags"] & oracle.FLAG_HIT
    assert np.array_equal(hit > 0, np.isfinite(expected))


# ---------------------------------------------------------------------------
# P2: constant cube -> slab law, for every ray and camera; ERT closed form
# ---------------------------------------------------------------------------
def random_poses(seed, N, count):
    rng = np.random.default_rng(seed)
    c = (np.asarray(N) - 1) / 2.0
    out = []
    for _ in range(count):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        R = rng.uniform(1.2, 3.0) * np.linalg.norm(N) / 2
        tgt = c + rng.uniform(-2, 2, size=3)
        out.append(synth.Camera(eye=tuple(c + R * d), target=tuple(tgt), up=(0.3, 0.2, 1.0),
                                fovy_deg=float(rng.uniform(20, 70))))
    return out


@pytest.mark.parametrize("pose", range(4))
def test_p2_constant_cube_slab_law(pose):
    N = (20, 24, 28)
    v = 7.3
    vol = np.full(N[::-1], v, dtype=np.float64)
    v0, v1, kmax = 2.0, 12.0, 0.8
    tf = ramp64(256, kmax)
    s = (v - v0) / (v1 - v0)
    kappa, rgb = kmax * s, np.array([s, 0.5 * s, 1.0 - s])
    cam = random_poses(100 + pose, N, 4)[pose]
    W, H = 23, 17
    res = oracle.render(vol, mode=oracle.EA, tf=tf, v0=v0, v1=v1, camera=cam, width=W, height=H,
                        step=0.37, ert=2.0)
    img = res["image"]
    nhit = 0
    for j in range(H):
        for i in range(W):
            o, d = oracle.pixel_ray(cam, W, H, i, j)
            ch = face_clip_chord(o, d, N, False)
            if ch is None:
                assert np.all(img[j, i] == 0.0) or np.max(np.abs(img[j, i])) < 1e-9
                continue
            nhit += 1
            L = ch[1] - ch[0]
            A = 1.0 - math.exp(-kappa * L)
            assert abs(img[j, i, 3] - A) < 1e-12
            assert np.max(np.abs(img[j, i, :3] - rgb * A)) < 1e-12
            assert res["n_nominal"][j, i] == math.ceil(L / 0.37 - 1e-12)
    assert nhit > 20


def test_p2_constant_cube_ert_stop_index():
    N = (16, 16, 200)
    v = 9.0
    vol = np.full(N[::-1], v, dtype=np.float64)
    v0, v1, kmax = 3.0, 20.0, 0.3
    tf = ramp64(256, kmax)
    s = (v - v0) / (v1 - v0)
    kappa = kmax * s
    W, H = 8, 8
    cam = synth.axis_camera(*N, "z", W, H)
    a = 0.95
    step = 0.5
    res = oracle.render(vol, mode=oracle.EA, tf=tf, v0=v0, v1=v1, camera=cam, width=W, height=H,
                        step=step, ert=a)
    m = math.ceil(math.log(1.0 / (1.0 - a)) / (kappa * step))
    assert m < 400
    A = 1.0 - math.exp(-kappa * m * step)
    assert np.all(res["n_exec"] == m)
    assert np.allclose(res["image"][..., 3], A, rtol=0, atol=1e-13)
    assert np.allclose(res["image"][..., 0], s * A, rtol=0, atol=1e-13)
    assert np.all(res["flags"] & oracle.FLAG_ERT_STOPPED)


# ---------------------------------------------------------------------------
# P3: trilinear reproduces multilinear fields exactly (single-sample rays)
# ---------------------------------------------------------------------------
def test_p3_trilinear_reproduces_multilinear_field():
    N = (9, 11, 13)
    rng = np.random.default_rng(3)
    c = rng.uniform(-2, 2, size=8)

    def field(x, y, z):
        return (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z + c[6] * x * z
                + c[7] * x * y * z)

    z, y, x = np.meshgrid(np.arange(N[2]), np.arange(N[1]), np.arange(N[0]), indexing="ij")
    vol = field(x.astype(float), y.astype(float), z.astype(float))
    checked = 0
    for cam in random_poses(7, N, 6):
        W, H = 15, 15
        # a step longer than any chord gives one sample, at the chord midpoint
        res = oracle.render(vol, mode=oracle.MIP, interp=oracle.TRILINEAR, camera=cam, width=W,
                            height=H, step=1e6)
        for j in range(H):
            for i in range(W):
                o, d = oracle.pixel_ray(cam, W, H, i, j)
                ch = face_clip_chord(o, d, N, False)
                if ch is None:
                    continue
                p = o + 0.5 * (ch[0] + ch[1]) * d
                if np.all(p >= 0) and np.all(p <= np.asarray(N) - 1):
                    exp = field(*p)
                    assert abs(res["image"][j, i] - exp) < 1e-11 * max(1.0, abs(exp))
                    checked += 1
    assert checked > 100


def test_p3_nearest_single_sample_picks_rounded_voxel():
    N = (9, 11, 13)
    rng = np.random.default_rng(4)
    vol = rng.normal(size=N[::-1])
    checked = 0
    for cam in random_poses(8, N, 4):
        W, H = 15, 15
        res = oracle.render(vol, mode=oracle.MIP, interp=oracle.NEAREST, camera=cam, width=W,
                            height=H, step=1e6)
        for j in range(H):
            for i in range(W):
                o, d = oracle.pixel_ray(cam, W, H, i, j)
                ch = face_clip_chord(o, d, N, False)
                if ch is None:
                    continue
                p = o + 0.5 * (ch[0] + ch[1]) * d
                k = [min(max(int(math.floor(p[a] + 0.5)), 0), N[a] - 1) for a in range(3)]
                assert res["image"][j, i] == vol[k[2], k[1], k[0]]
                checked += 1
    assert checked > 100


# ---------------------------------------------------------------------------
# P4: zero extinction / clip above the data -> zero image
# ---------------------------------------------------------------------------
def test_p4_zero_kappa_and_high_clip_give_zero_image(tiny_cube):
    nz, ny, nx = tiny_cube.shape
    cam = synth.orbit_camera(nx, ny, nz, 0.7, 0.3)
    tf = ramp64(256, 1.0)
    tf0 = tf.copy()
    tf0[:, 3] = 0.0
    r = oracle.render(tiny_cube, mode=oracle.EA, tf=tf0, v0=3, v1=20, camera=cam, width=48,
                      height=40)
    assert np.all(r["image"] == 0.0)
    gmax = float(tiny_cube.max())
    r = oracle.render(tiny_cube, mode=oracle.EA, tf=tf, v0=3, v1=20, clip=gmax + 1e-3, camera=cam,
                      width=48, height=40)
    assert np.all(r["image"] == 0.0)
    r = oracle.render(tiny_cube, mode=oracle.MIP, clip=gmax + 1e-3, camera=cam, width=48, height=40)
    img = r["image"]
    hit = (r["flags"] & oracle.FLAG_HIT) > 0
    assert np.all(img[hit] == 0.0) and np.all(img[~hit] == -INF)
    assert hit.sum() > 100


# ---------------------------------------------------------------------------
# P5: a single bright voxel lights its pinhole projection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(3))
def test_p5_single_voxel_footprint_matches_projection(seed):
    rng = np.random.default_rng(seed)
    N = (16, 18, 20)
    vol = np.zeros(N[::-1])
    kx, ky, kz = rng.integers(3, 13, size=3)
    vol[kz, ky, kx] = 10.0
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    cam = synth.Camera(eye=tuple(np.array([kx, ky, kz]) + 30 * d), target=(7.5, 8.5, 9.5),
                       up=(0, 0, 1), fovy_deg=40.0)
    W, H = 161, 121
    res = oracle.render(vol, mode=oracle.MIP, interp=oracle.NEAREST, camera=cam, width=W, height=H,
                        step=0.05)
    lit = res["image"] > 0
    f, r, u = basis(cam)
    h = math.tan(math.radians(cam.fovy_deg) / 2)
    a = W / H

    def project(p):
        q = np.asarray(p, dtype=float) - np.asarray(cam.eye)
        zc = q @ f
        xn, yn = (q @ r) / (zc * h * a), (q @ u) / (zc * h)
        return (xn + 1) / 2 * W - 0.5, (1 - yn) / 2 * H - 0.5

    ci, cj = project((kx, ky, kz))
    corners = [project((kx + sx * 0.5, ky + sy * 0.5, kz + sz * 0.5)) for sx in (-1, 1)
               for sy in (-1, 1) for sz in (-1, 1)]
    ii = [c[0] for c in corners]
    jj = [c[1] for c in corners]
    js, is_ = np.nonzero(lit)
    assert lit.sum() > 4
    assert is_.min() >= math.floor(min(ii)) and is_.max() <= math.ceil(max(ii))
    assert js.min() >= math.floor(min(jj)) and js.max() <= math.ceil(max(jj))
    assert lit[int(round(cj)), int(round(ci))]


# ---------------------------------------------------------------------------
# Front-to-back order: two slabs along the view axis
# ---------------------------------------------------------------------------
def test_two_slab_front_to_back_over():
    N = (8, 8, 64)
    va, vb = 6.0, 14.0
    vol = np.empty(N[::-1])
    vol[:32] = va
    vol[32:] = vb
    v0, v1 = 2.0, 20.0
    tf = ramp64(256, 0.5)
    cam = synth.axis_camera(*N, "z", 8, 8)  # looks along +z: slab a is in front
    res = oracle.render(vol, mode=oracle.EA, interp=oracle.NEAREST, tf=tf, v0=v0, v1=v1, camera=cam,
                        width=8, height=8, step=0.5, ert=2.0)

    def layer(v, L):
        s = (v - v0) / (v1 - v0)
        A = 1 - math.exp(-0.5 * s * L)
        return np.array([s, 0.5 * s, 1 - s]) * A, A

    ca, Aa = layer(va, 32.0)
    cb, Ab = layer(vb, 32.0)
    C = ca + (1 - Aa) * cb
    A = 1 - (1 - Aa) * (1 - Ab)
    img = res["image"]
    assert np.allclose(img[..., :3], C, atol=1e-12, rtol=0)
    assert np.allclose(img[..., 3], A, atol=1e-12, rtol=0)
    # swapping the slabs changes the colour: order matters
    cam2 = synth.Camera(eye=(3.5, 3.5, 200.0), target=cam.target, up=(0, 1, 0), ortho=True,
                        ortho_w=cam.ortho_w, ortho_h=cam.ortho_h)
    res2 = oracle.render(vol, mode=oracle.EA, interp=oracle.NEAREST, tf=tf, v0=v0, v1=v1,
                         camera=cam2, width=8, height=8, step=0.5, ert=2.0)
    C2 = cb + (1 - Ab) * ca
    assert np.allclose(res2["image"][..., :3], C2, atol=1e-12, rtol=0)
    assert np.max(np.abs(C2 - C)) > 1e-2


# ---------------------------------------------------------------------------
# Transfer-function interpolation equals numpy's piecewise-linear interp
# ---------------------------------------------------------------------------
def test_tf_rows_interpolate_like_numpy_interp():
    rng = np.random.default_rng(12)
    n = 17
    tf = rng.uniform(0, 1, size=(n, 4))
    v0, v1 = -1.5, 4.0
    N = (4, 4, 4)
    cam = synth.axis_camera(*N, "z", 1, 1)
    for v in [-3.0, -1.5, -0.2, 0.0, 1.1, 2.7, 3.999, 4.0, 9.0]:
        vol = np.full(N[::-1], v)
        res = oracle.render(vol, mode=oracle.EA, tf=tf, v0=v0, v1=v1, camera=cam, width=1,
                            height=1, step=0.5, ert=2.0)
        u = np.clip((v - v0) / (v1 - v0) * (n - 1), 0, n - 1)
        row = [np.interp(u, np.arange(n), tf[:, c]) for c in range(4)]
        L = 4.0
        A = 1 - math.exp(-row[3] * L)
        assert abs(res["image"][0, 0, 3] - A) < 1e-12
        assert np.allclose(res["image"][0, 0, :3], np.array(row[:3]) * A, atol=1e-12, rtol=0)


def test_clip_zeroes_samples_below_threshold():
    # left half of the columns below the clip, right half above: only the right half renders
    N = (8, 4, 16)
    vol = np.empty(N[::-1])
    vol[..., :4] = 4.0
    vol[..., 4:] = 6.0
    tf = ramp64(256, 1.0)
    cam = synth.axis_camera(*N, "z", 8, 4)
    res = oracle.render(vol, mode=oracle.EA, interp=oracle.NEAREST, tf=tf, v0=0.0, v1=10.0,
                        clip=5.0, camera=cam, width=8, height=4, step=0.5, ert=2.0)
    img = res["image"]
    assert np.all(img[:, :4] == 0.0)
    A = 1 - math.exp(-0.6 * 16)
    assert np.allclose(img[:, 4:, 3], A, atol=1e-12, rtol=0)


# ---------------------------------------------------------------------------
# P10: second-order convergence to the continuous emission-absorption integral
# ---------------------------------------------------------------------------
def test_p10_midpoint_rule_converges_to_continuous_integral():
    from scipy import integrate
    N = (4, 4, 40)
    g0, g1 = 3.0, 15.0  # value rises linearly along z from g0 (z=0) to g1 (z=N-1)
    z = np.arange(N[2], dtype=float)
    col = g0 + (g1 - g0) * z / (N[2] - 1)
    vol = np.broadcast_to(col[:, None, None], N[::-1]).copy()
    v0, v1, kmax = 0.0, 20.0, 0.6
    tf = ramp64(256, kmax)

    def vz(zz):  # clamp-to-edge field along the ray
        q = min(max(zz, 0.0), N[2] - 1)
        return g0 + (g1 - g0) * q / (N[2] - 1)

    def kap(zz):
        return kmax * vz(zz) / v1

    def rgb(zz, c):
        s = vz(zz) / v1
        return (s, 0.5 * s, 1 - s)[c]

    a, b = -0.5, N[2] - 0.5
    Z = N[2] - 1.0

    def tau(zz):  # optical depth from the entry face, integrated in closed form
        if zz <= 0.0:
            I = g0 * (zz + 0.5)
        elif zz <= Z:
            I = 0.5 * g0 + g0 * zz + (g1 - g0) * zz * zz / (2 * Z)
        else:
            I = 0.5 * g0 + g0 * Z + (g1 - g0) * Z / 2 + g1 * (zz - Z)
        return kmax / v1 * I

    exact = [integrate.quad(lambda zz, c=c: rgb(zz, c) * kap(zz) * math.exp(-tau(zz)), a, b,
                            points=[0.0, Z], limit=400, epsabs=1e-14, epsrel=1e-13)[0]
             for c in range(3)]
    exact_alpha = 1 - math.exp(-tau(b))
    cam = synth.axis_camera(*N, "z", 1, 1)
    errs = []
    # steps 0.5/m put the clamp kinks (z = 0 and z = N-1) on segment boundaries, so the
    # extinction is linear inside every segment: midpoints integrate it exactly, and the colour
    # integral converges at second order
    for step in [0.5, 0.25, 0.125, 0.0625]:
        res = oracle.render(vol, mode=oracle.EA, tf=tf, v0=v0, v1=v1, camera=cam, width=1, height=1,
                            step=step, ert=2.0)
        px = res["image"][0, 0]
        errs.append(max(abs(px[c] - exact[c]) for c in range(3)))
        assert abs(px[3] - exact_alpha) < 1e-12
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.5 < e0 / e1 < 4.5, errs  # second order: a factor 4 per halving


# ---------------------------------------------------------------------------
# P7 and P8: early termination bound, mirror symmetry
# ---------------------------------------------------------------------------
def test_p7_ert_changes_image_by_at_most_remaining_transmittance(tiny_cube):
    nz, ny, nx = tiny_cube.shape
    cam = synth.orbit_camera(nx, ny, nz, 1.1, 0.4)
    tf = ramp64(256, 8.0)  # opaque enough that bright sources terminate rays early
    kw = dict(mode=oracle.EA, tf=tf, v0=3.0, v1=20.0, clip=3.0, camera=cam, width=64, height=64)
    on = oracle.render(tiny_cube, ert=0.99, **kw)
    off = oracle.render(tiny_cube, ert=2.0, **kw)
    d = np.abs(on["image"] - off["image"])
    assert d.max() <= 0.01 + 1e-12
    stopped = (on["flags"] & oracle.FLAG_ERT_STOPPED) > 0
    assert stopped.sum() > 0
    assert np.all(on["image"][stopped][:, 3] >= 0.99)
    assert np.all(on["n_exec"][stopped] <= on["n_nominal"][stopped])
    assert np.all(on["n_exec"][~stopped] == on["n_nominal"][~stopped])
    assert (on["n_exec"] < on["n_nominal"]).sum() > 0


def test_p8_mirror_cube_and_camera_mirrors_image(tiny_cube):
    nz, ny, nx = tiny_cube.shape
    vol = tiny_cube[:, :20, :24].astype(np.float64).copy()
    nz, ny, nx = vol.shape
    cam = synth.Camera(eye=(-30.0, 50.0, 90.0), target=(10.0, 9.0, 60.0), up=(0.1, 0.0, 1.0),
                       fovy_deg=35.0)
    mir = lambda p: ((nx - 1) - p[0], p[1], p[2])
    cam2 = synth.Camera(eye=mir(cam.eye), target=mir(cam.target), up=(-cam.up[0], cam.up[1],
                                                                     cam.up[2]), fovy_deg=35.0)
    tf = ramp64(256, 1.0)
    for mode in (oracle.EA, oracle.MIP):
        kw = dict(mode=mode, tf=tf, v0=0.0, v1=8.0, width=40, height=30, ert=2.0)
        a = oracle.render(vol, camera=cam, **kw)["image"]
        b = oracle.render(vol[:, :, ::-1], camera=cam2, **kw)["image"]
        fin = np.isfinite(a)
        assert np.array_equal(fin, np.isfinite(b[:, ::-1]))
        assert np.allclose(a[fin], b[:, ::-1][fin], atol=1e-10, rtol=0)


# ---------------------------------------------------------------------------
# Ambiguity flags: nearest ties and grazing rays are reported
# ---------------------------------------------------------------------------
def test_nearest_tie_is_flagged():
    N = (4, 4, 4)
    vol = np.arange(64, dtype=np.float64).reshape(4, 4, 4)
    # an orthographic 4x4 window of width 4 puts pixel centres on integers: no tie in x/y;
    # a window of width 3 over 3 pixels puts them at -0.5..: here use centres at k + 1/2
    cam = synth.Camera(eye=(1.0, 1.5, -10), target=(1.0, 1.5, 1.5), up=(0, -1, 0), ortho=True,
                       ortho_w=4.0, ortho_h=4.0)
    res = oracle.render(vol, mode=oracle.MIP, interp=oracle.NEAREST, camera=cam, width=4, height=4)
    # columns sit at x = i - 1/2: ties between voxels i-1 and i for i >= 1 (at x = -1/2 both
    # candidates clamp to voxel 0, so there is no ambiguity there)
    fl = res["flags"]
    assert np.all(fl & oracle.FLAG_HIT)
    assert np.all(fl[:, 1:] & oracle.FLAG_NEAREST_AMBIG)


# ---------------------------------------------------------------------------
# 16-bit storage: exact decoding, round-to-nearest-even encoding
# ---------------------------------------------------------------------------
def test_f16_decode_matches_numpy_for_all_codes():
    L = oracle.lib()
    codes = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    ref = codes.view(np.float16).astype(np.float64)
    got = np.array([L.orc_decode_f16(int(c)) for c in codes])
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.isnan(got), np.isnan(ref))


def test_bf16_encode_decode_match_torch():
    import torch
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 20, 200000), rng.normal(0, 1e-3, 1000),
                        [0.0, -0.0, 1.0, 3.0, 50.0, 1e-40, -1e-40, 65504.0, 70000.0]]).astype(np.float32)
    # force exact ties: values whose low 16 mantissa bits are 0x8000
    t = ((rng.integers(0, 2**7, 500).astype(np.uint32) << 16) | 0x3F808000).view(np.float32)
    x = np.concatenate([x, t, -t])
    ours = oracle.to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    dec = oracle.decode_bits(ours, oracle.BF16)
    refd = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(dec, refd)
    L = oracle.lib()
    assert all(L.orc_decode_bf16(int(c)) == d for c, d in zip(ours[:2000], dec[:2000]))


def test_f16_encode_matches_torch():
    import torch
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(0, 30, 100000), rng.normal(0, 1e-5, 1000)]).astype(np.float32)
    ours = oracle.to_f16_bits(x)
    ref = torch.from_numpy(x).to(torch.float16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_storage_decode_in_renderer_matches_promoted_values(tiny_cube):
    """Rendering 16-bit codes with a scale equals rendering their decoded float64 values."""
    nz, ny, nx = tiny_cube.shape
    cam = synth.orbit_camera(nx, ny, nz, 2.0, -0.2)
    tf = ramp64(256, 1.0)
    for dt, enc in ((oracle.F16, oracle.to_f16_bits), (oracle.BF16, oracle.to_bf16_bits)):
        bits = enc(tiny_cube / 2.0)
        dec = oracle.decode_bits(bits, dt) * 2.0
        kw = dict(mode=oracle.EA, tf=tf, v0=3, v1=20, clip=3, camera=cam, width=32, height=32)
        a = oracle.render(bits, vox_dtype=dt, vox_scale=2.0, **kw)["image"]
        b = oracle.render(dec, **kw)["image"]
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Ambiguity flags pinned by constructed rays: each flag is raised exactly when
# the quantity it watches lies within its margin of the decision threshold.
# ---------------------------------------------------------------------------
def _flat_tf(kappa):
    """Two equal rows: extinction kappa and grey colour for every value."""
    return np.array([[0.5, 0.5, 0.5, kappa], [0.5, 0.5, 0.5, kappa]], dtype=np.float64)


@pytest.mark.parametrize("delta,flagged,stop", [(0.5e-5, True, 41), (2e-5, False, 41),
                                                (-0.5e-5, True, 40), (-2e-5, False, 40)])
def test_ert_flag_margin(delta, flagged, stop):
    """Constant cube, rays along z: after k full segments of length 0.5 the
    opacity is 1 - exp(-0.05 * 0.5 k) (closed form).  The early-termination
    threshold is put delta away from the opacity after 40 samples: the ERT
    flag is raised iff |delta| < amb_ert (1e-5), and the ray stops after
    sample 40 (delta <= 0) or 41 (delta > 0)."""
    N = (8, 8, 64)
    vol = np.full(N[::-1], 0.5, dtype=np.float64)
    a40 = -math.expm1(-0.05 * 0.5 * 40)
    cam = synth.axis_camera(*N, "z", 4, 4)
    res = oracle.render(vol, mode=oracle.EA, tf=_flat_tf(0.05), v0=0.0, v1=1.0, camera=cam,
                        width=4, height=4, step=0.5, ert=a40 + delta, amb_ert=1e-5)
    fl = res["flags"]
    assert np.all(fl & oracle.FLAG_ERT_STOPPED)
    assert np.all(res["n_exec"] == stop)
    assert np.all(((fl & oracle.FLAG_ERT_AMBIG) > 0) == flagged)
    assert np.allclose(res["image"][..., 3], -math.expm1(-0.05 * 0.5 * stop), rtol=0, atol=1e-12)


@pytest.mark.parametrize("rel,flagged", [(0.5e-4, True), (-0.5e-4, True), (2e-4, False),
                                         (-2e-4, False)])
def test_clip_flag_margin(rel, flagged):
    """A transfer function with a jump at the clip (kappa(clip) > 0): a constant
    cube whose value lies rel * max(1, |clip|) from the clip is flagged iff
    |rel| < amb_clip (1e-4).  Below the clip the image is exactly zero; above
    it, the slab law holds."""
    N = (6, 6, 10)
    clip = 3.0
    v = clip + rel * clip
    vol = np.full(N[::-1], v, dtype=np.float64)
    cam = synth.axis_camera(*N, "z", 3, 3)
    res = oracle.render(vol, mode=oracle.EA, tf=_flat_tf(0.2), v0=0.0, v1=10.0, clip=clip,
                        camera=cam, width=3, height=3, step=0.5, ert=2.0, amb_clip=1e-4)
    fl = res["flags"]
    assert np.all(((fl & oracle.FLAG_CLIP_AMBIG) > 0) == flagged)
    A = res["image"][..., 3]
    if rel < 0:
        assert np.all(res["image"] == 0.0)
    else:
        assert np.allclose(A, -math.expm1(-0.2 * 10.0), rtol=0, atol=1e-12)


def test_clip_flag_absent_when_transfer_function_is_continuous_at_clip():
    """With the ramp starting at the clip (kappa(clip) = 0) the result is
    continuous there: a cube exactly at the clip is not flagged and renders
    to zero."""
    N = (6, 6, 10)
    vol = np.full(N[::-1], 3.0, dtype=np.float64)
    cam = synth.axis_camera(*N, "z", 3, 3)
    res = oracle.render(vol, mode=oracle.EA, tf=ramp64(), v0=3.0, v1=20.0, clip=3.0, camera=cam,
                        width=3, height=3, step=0.5, ert=2.0)
    assert not np.any(res["flags"] & oracle.FLAG_CLIP_AMBIG)
    assert np.all(res["image"] == 0.0)


@pytest.mark.parametrize("chord,flagged", [(0.5e-6, True), (4e-6, False)])
def test_graze_flag_margin(chord, flagged):
    """An orthographic ray along (1, 1, 0)/sqrt(2) that cuts the box's edge at
    x = N-1/2, y = -1/2: starting on the face y = -1/2 at x = N - 1/2 - a, its
    chord is a*sqrt(2) (closed form).  The graze flag is raised iff the chord
    is below amb_graze (1e-6)."""
    N = (8, 8, 8)
    a = chord / math.sqrt(2.0)
    d = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    target = np.array([N[0] - 0.5 - a, -0.5, 3.5])
    cam = synth.Camera(eye=tuple(target - 10.0 * d), target=tuple(target), up=(0, 0, 1),
                       ortho=True, ortho_w=1.0, ortho_h=1.0)
    vol = np.full(N[::-1], 1.0, dtype=np.float64)
    res = oracle.render(vol, mode=oracle.MIP, camera=cam, width=1, height=1, step=0.5,
                        amb_graze=1e-6)
    o, dd = oracle.pixel_ray(cam, 1, 1, 0, 0)
    hit, t0, t1 = oracle.slab(N[::-1], cam, 1, 1, o, dd)
    assert hit and abs((t1 - t0) - chord) < 1e-12
    fl = int(res["flags"][0, 0])
    assert fl & oracle.FLAG_HIT
    assert bool(fl & oracle.FLAG_GRAZE_AMBIG) == flagged


def test_nearest_tie_bounds_are_the_candidate_maxima():
    """Pixel centres on voxel faces (ties in x): the reference's bounds of the
    correct maxima equal a brute force over both candidate voxels of every
    tied coordinate; untied pixels have bounds equal to the value."""
    N = (4, 4, 4)
    vol = np.arange(64, dtype=np.float64).reshape(4, 4, 4)
    cam = synth.Camera(eye=(1.0, 1.5, -10), target=(1.0, 1.5, 1.5), up=(0, -1, 0), ortho=True,
                       ortho_w=4.0, ortho_h=4.0)
    res = oracle.render(vol, mode=oracle.MIP, interp=oracle.NEAREST, camera=cam, width=4, height=4)
    img, b, fl = res["image"], res["bounds"], res["flags"]

    def cands(x, n):
        s = x + 0.5
        k = math.floor(s)
        fr = s - k
        out = {k}
        if 0.0 < s < n and (fr < 1e-6 or fr > 1.0 - 1e-6):
            out.add(k - 1 if fr < 0.5 else k + 1)
        return sorted(min(max(c, 0), n - 1) for c in out)

    ntie = 0
    for j in range(4):
        for i in range(4):
            o, d = oracle.pixel_ray(cam, 4, 4, i, j)
            X, Y = cands(o[0], 4), cands(o[1], 4)
            # samples along z sit at -1/4 + k/2: never a tie; the maximum is at z = 3
            lo = max(min(vol[z, y, x] for x in X for y in Y) for z in range(4))
            hi = max(max(vol[z, y, x] for x in X for y in Y) for z in range(4))
            assert b[j, i, 0] == lo and b[j, i, 1] == hi
            assert lo <= img[j, i] <= hi
            tie = bool(fl[j, i] & oracle.FLAG_NEAREST_AMBIG)
            assert tie == (len(X) > 1 or len(Y) > 1)
            ntie += tie
            if not tie:
                assert lo == hi == img[j, i]
    assert ntie >= 8


# ---------------------------------------------------------------------------
# Sub-cube partials (Sec. 3.1, process steps 1, 4 and 5): windows along one
# axis that tile it partition every ray's lattice; "over" of the EA partials in
# visibility order and the maximum of the MIP partials give the whole image.
# ---------------------------------------------------------------------------
def _windows(n, cuts):
    edges = [-np.inf] + [c - 0.5 for c in cuts] + [np.inf]
    return list(zip(edges[:-1], edges[1:]))


def test_subcube_partials_partition_and_compose():
    spec = synth.CubeSpec(30, 26, 40, seed=77, sources=synth.SourcePop(4, 5, 20, False, 2, 5, 2, 6))
    vol = synth.cube(spec)
    tf = synth.ramp_tf(64, 1.0).astype(np.float64)
    # eye below the cube along z: every ray that hits it moves up in z
    cam = synth.Camera(eye=(14.0, -20.0, -45.0), target=(14.5, 12.5, 19.5), up=(0.0, 0.0, 1.0),
                       fovy_deg=50.0)
    common = dict(tf=tf, v0=3.0, v1=20.0, clip=3.0, step=0.5, ert=2.0, camera=cam, width=40,
                  height=36)
    whole = oracle.render(vol, mode=oracle.EA, **common)
    wins = _windows(40, [7, 19, 32])
    parts = [oracle.render(vol, mode=oracle.EA, window=(2, lo, hi), **common) for lo, hi in wins]
    assert np.array_equal(sum(p["n_nominal"] for p in parts), whole["n_nominal"])
    comp = oracle.composite_over([p["image"] for p in parts])
    assert np.max(np.abs(comp - whole["image"])) < 1e-12
    # back-to-front order is not the same image where partials overlap on a ray
    wrong = oracle.composite_over([p["image"] for p in parts[::-1]])
    assert np.max(np.abs(wrong - whole["image"])) > 1e-3
    mwhole = oracle.render(vol, mode=oracle.MIP, **common)
    mparts = [oracle.render(vol, mode=oracle.MIP, window=(2, lo, hi), **common)["image"] for lo, hi in wins]
    assert np.array_equal(oracle.composite_max(mparts), mwhole["image"])


def test_subcube_window_edges_are_flagged():
    vol = np.zeros((8, 8, 8), np.float32)
    cam = synth.axis_camera(8, 8, 8, "z", 8, 8)
    # samples along z sit at -0.25 + 0.5k: a window edge at 1.75 meets one exactly
    r = oracle.render(vol, mode=oracle.MIP, camera=cam, width=8, height=8, step=0.5,
                      window=(2, -np.inf, 1.75))
    assert np.all((r["flags"] & oracle.FLAG_WINDOW_AMBIG) > 0)
    r = oracle.render(vol, mode=oracle.MIP, camera=cam, width=8, height=8, step=0.5,
                      window=(2, -np.inf, 1.5))
    assert not np.any((r["flags"] & oracle.FLAG_WINDOW_AMBIG) > 0)
    assert np.all(r["n_nominal"] == 4)
