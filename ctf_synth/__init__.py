"""Seeded synthetic inputs shared by the CPU oracle and the HIP library.

This module holds no part of the filtering method: it only draws the inputs
both sides consume (screen-space texture coordinates and their derivatives,
the random parameters of the procedural texture, and the initial decoder
parameters).  Every array it returns is plain numpy; nothing here is
imported by ``oracle/`` or by the HIP binding, the tests and the benchmark
call it and hand the same buffers to both sides.

Geometry follows the paper's evaluation setup (supplement S3, "Scenes and
Textures"): textured planes seen through a pinhole camera, spanning strong
magnification to minification.  The paper's photographic textures are not
available; the procedural sinusoid texture stands in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Plane", "Scene", "sinusoid_params", "affine_params", "plane_scene",
    "tilted_plane_scene", "random_planes_scene", "layer_transform",
    "magnifying_fraction", "texel_ratio", "decoder_init", "decoder_layout",
    "head_on_quad_uv",
]


# ---------------------------------------------------------------------------
# procedural texture parameters
# ---------------------------------------------------------------------------

def sinusoid_params(width: int, n_terms: int, max_freq: int, seed: int):
    """Random parameters of the sum-of-sinusoids texture.

    Per channel c and term k: integer spatial frequencies (p, q) in
    [-F, F]^2, not both zero; integer phase j in [0, W); amplitude a > 0,
    normalised so that sum_k a = 1 for every channel.  Amplitudes are stored
    as float32 and both sides read exactly those float32 values.

    Returns (pqj int32 [4][K][3], amp float32 [4][K]).
    """
    if width <= 0 or width & (width - 1):
        raise ValueError("texture width must be a power of two")
    rng = np.random.default_rng(np.random.SeedSequence([0x51A, seed]))
    pqj = np.zeros((4, n_terms, 3), dtype=np.int32)
    amp = np.zeros((4, n_terms), dtype=np.float64)
    for c in range(4):
        for k in range(n_terms):
            while True:
                p, q = rng.integers(-max_freq, max_freq + 1, size=2)
                if p != 0 or q != 0:
                    break
            pqj[c, k] = (p, q, rng.integers(0, width))
        a = rng.uniform(0.5, 1.5, size=n_terms)
        amp[c] = a / a.sum()
    return pqj, amp.astype(np.float32)


def affine_params(seed: int) -> np.ndarray:
    """Random affine texture f_c(x, y) = c0 + c1*x + c2*y, float64 [4][3]."""
    rng = np.random.default_rng(np.random.SeedSequence([0xAFF, seed]))
    coef = np.empty((4, 3))
    coef[:, 0] = rng.uniform(-1, 1, 4)
    coef[:, 1:] = rng.uniform(-0.05, 0.05, (4, 2))
    return coef


# ---------------------------------------------------------------------------
# scenes: planes under a pinhole camera
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Plane:
    origin: np.ndarray      # a point on the plane (world), where uv = offset
    e1: np.ndarray          # in-plane unit axis -> u
    e2: np.ndarray          # in-plane unit axis -> v
    size: float             # world length of one texture repeat
    offset: Tuple[float, float] = (0.0, 0.0)

    @property
    def normal(self):
        return np.cross(self.e1, self.e2)


@dataclasses.dataclass
class Scene:
    width: int
    height: int
    uv: np.ndarray          # float32 [H][W][2]; NaN where no surface
    duv: np.ndarray         # float32 [H][W][4] = (du/dx, dv/dx, du/dy, dv/dy)
    info: dict


def _rays(width, height, fov_y_deg):
    th = math.tan(math.radians(fov_y_deg) / 2)
    aspect = width / height
    px = (np.arange(width) + 0.5)
    py = (np.arange(height) + 0.5)
    x = (2 * px / width - 1) * th * aspect
    y = (1 - 2 * py / height) * th
    X, Y = np.meshgrid(x, y)
    d = np.stack([X, Y, -np.ones_like(X)], axis=-1)
    ddx = np.array([2 * th * aspect / width, 0.0, 0.0])
    ddy = np.array([0.0, -2 * th / height, 0.0])
    return d, ddx, ddy


def _hit(plane: Plane, d, ddx, ddy):
    """Ray/plane hit distance and analytic uv, d(uv)/dpixel (all float64)."""
    n = plane.normal
    on = float(plane.origin @ n)
    dn = d @ n
    with np.errstate(divide="ignore", invalid="ignore"):
        lam = on / dn
    valid = np.isfinite(lam) & (lam > 0)
    P = lam[..., None] * d
    rel = P - plane.origin
    u = rel @ plane.e1 / plane.size + plane.offset[0]
    v = rel @ plane.e2 / plane.size + plane.offset[1]
    out = [u, v]
    for dd in (ddx, ddy):
        ddn = float(dd @ n)
        dlam = -on * ddn / (dn * dn)
        dP = dlam[..., None] * d + lam[..., None] * dd
        out.append(dP @ plane.e1 / plane.size)
        out.append(dP @ plane.e2 / plane.size)
    u, v, dudx, dvdx, dudy, dvdy = out
    return lam, valid, np.stack([u, v], -1), np.stack([dudx, dvdx, dudy, dvdy], -1)


def plane_scene(planes: Sequence[Plane], width: int, height: int, fov_y_deg: float,
                info: Optional[dict] = None) -> Scene:
    """Render uv and uv derivatives of the nearest plane hit per pixel.

    Computed in float64 and stored as float32.  Pixels hitting no plane get
    NaN uv (and NaN derivatives): such pixels are inactive.
    """
    d, ddx, ddy = _rays(width, height, fov_y_deg)
    best = np.full((height, width), np.inf)
    uv = np.full((height, width, 2), np.nan)
    duv = np.full((height, width, 4), np.nan)
    for pl in planes:
        lam, valid, puv, pduv = _hit(pl, d, ddx, ddy)
        take = valid & (lam < best)
        best = np.where(take, lam, best)
        uv[take] = puv[take]
        duv[take] = pduv[take]
    return Scene(width, height, uv.astype(np.float32), duv.astype(np.float32),
                 dict(info or {}))


def texel_ratio(duv: np.ndarray, tex_w: int, tex_h: int) -> np.ndarray:
    """Texels per pixel (largest screen-axis footprint), float64, NaN-propagating.

    Used only to tune scene scales; the method makes its own decision.
    """
    a = duv[..., 0].astype(np.float64) * tex_w
    b = duv[..., 1].astype(np.float64) * tex_h
    c = duv[..., 2].astype(np.float64) * tex_w
    e = duv[..., 3].astype(np.float64) * tex_h
    return np.sqrt(np.maximum(a * a + b * b, c * c + e * e))


def magnifying_fraction(scene: Scene, tex_w: int, tex_h: int) -> float:
    r = texel_ratio(scene.duv, tex_w, tex_h)
    act = np.isfinite(scene.uv).all(-1)
    if not act.any():
        return 0.0
    return float(((r <= 1.0) & act).sum() / act.sum())


def _tilted_plane(beta, size, phi=0.0, offset=(0.0, 0.0)):
    n = np.array([0.0, math.sin(beta), math.cos(beta)])
    a = np.array([1.0, 0.0, 0.0])
    b = np.cross(n, a)
    c, s = math.cos(phi), math.sin(phi)
    e1 = c * a + s * b
    e2 = -s * a + c * b
    return Plane(np.array([0.0, 0.0, -1.0]), e1, e2, size, offset)


def tilted_plane_scene(width=256, height=256, tex_w=64, tex_h=64, fov_y_deg=60.0,
                       rho_min=0.05, rho_max=2.0, phi=0.3,
                       offset=(0.123, 0.456)) -> Scene:
    """One plane tilted away from the camera so texels/pixel spans rho_min..rho_max.

    The tilt is solved so that the largest/smallest texel-per-pixel ratio over
    the screen equals rho_max/rho_min, with the horizon off screen; the
    texture repeat size then sets the smallest ratio to rho_min.
    """
    from scipy.optimize import brentq

    def spread(beta):
        sc = plane_scene([_tilted_plane(beta, 1.0, phi, offset)], width, height, fov_y_deg)
        r = texel_ratio(sc.duv, tex_w, tex_h)
        return float(np.nanmax(r) / np.nanmin(r))

    hmax = math.radians(90 - fov_y_deg / 2) - 1e-4
    beta = brentq(lambda b: spread(b) - rho_max / rho_min, 0.0, hmax, xtol=1e-12)
    sc = plane_scene([_tilted_plane(beta, 1.0, phi, offset)], width, height, fov_y_deg)
    r = texel_ratio(sc.duv, tex_w, tex_h)
    size = float(np.nanmin(r) / rho_min)
    info = dict(kind="tilted_plane", beta_rad=beta, repeat_size=size, phi=phi,
                fov_y_deg=fov_y_deg, rho_min=rho_min, rho_max=rho_max)
    return plane_scene([_tilted_plane(beta, size, phi, offset)], width, height,
                       fov_y_deg, info)


def _random_planes(seed: int, n_planes: int):
    rng = np.random.default_rng(np.random.SeedSequence([0x91A, seed]))
    planes = []
    for _ in range(n_planes):
        # normal within 75 degrees of the view axis (+z faces the camera)
        cos_max = math.cos(math.radians(75))
        cz = rng.uniform(cos_max, 1.0)
        az = rng.uniform(0, 2 * math.pi)
        sz = math.sqrt(1 - cz * cz)
        n = np.array([sz * math.cos(az), sz * math.sin(az), cz])
        t = np.array([1.0, 0, 0]) if abs(n[0]) < 0.9 else np.array([0, 1.0, 0])
        a = np.cross(n, t); a /= np.linalg.norm(a)
        b = np.cross(n, a)
        phi = rng.uniform(0, 2 * math.pi)
        e1 = math.cos(phi) * a + math.sin(phi) * b
        e2 = np.cross(n, e1)
        depth = rng.uniform(1.0, 4.0)
        ox, oy = rng.uniform(-0.6, 0.6, 2) * depth
        size = math.exp(rng.uniform(math.log(0.5), math.log(2.0)))
        off = tuple(rng.uniform(0, 1, 2))
        planes.append(Plane(np.array([ox, oy, -depth]), e1, e2, size, off))
    return planes


def random_planes_scene(width=1920, height=1080, tex_w=2048, tex_h=2048, seed=1,
                        n_planes=4, fov_y_deg=60.0, target_magnify=0.70,
                        tune_width=480, scale: Optional[float] = None) -> Scene:
    """Several seeded planes; nearest hit wins; no hit gives NaN uv.

    A single global texture-repeat scale is tuned (on a reduced-resolution
    render of the same camera, then rescaled) so that ``target_magnify`` of
    the active pixels at ``tune_width`` x proportional height... have at most
    one texel per pixel.  Pass ``scale`` to reuse a tuned value, e.g. to
    render the same world at another resolution.
    """
    from scipy.optimize import brentq
    base = _random_planes(seed, n_planes)

    def with_scale(k):
        return [Plane(p.origin, p.e1, p.e2, p.size * k, p.offset) for p in base]

    if scale is None:
        th = max(1, round(tune_width * height / width))
        # texel ratio scales with (1/k) and with (1/width): tune at full width
        # by rescaling the derivative magnitudes of the reduced render.
        def frac(logk):
            sc = plane_scene(with_scale(math.exp(logk)), tune_width, th, fov_y_deg)
            sc.duv = sc.duv * (tune_width / width)
            return magnifying_fraction(sc, tex_w, tex_h) - target_magnify
        scale = math.exp(brentq(frac, math.log(1e-4), math.log(1e4), xtol=1e-6))
    sc = plane_scene(with_scale(scale), width, height, fov_y_deg)
    sc.info = dict(kind="random_planes", seed=seed, n_planes=n_planes, scale=scale,
                   fov_y_deg=fov_y_deg, target_magnify=target_magnify,
                   magnify=magnifying_fraction(sc, tex_w, tex_h),
                   active=float(np.isfinite(sc.uv).all(-1).mean()))
    return sc


def layer_params(seed: int, layer: int):
    """Scale s_l ~ U[0.25, 4] and rotation theta_l ~ U[0, 2*pi) of material
    layer ``layer``, drawn from (seed, layer); M_l = s_l R(theta_l)."""
    rng = np.random.default_rng(np.random.SeedSequence([0x1A7, seed, layer]))
    s = rng.uniform(0.25, 4.0)
    th = rng.uniform(0, 2 * math.pi)
    M = s * np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    return s, th, M


def layer_transform(scene: Scene, seed: int, layer: int):
    """Per-layer uv: uv_l = R(theta_l) * s_l * uv, derivatives alike.

    Returns (uv float32, duv float32, s_l, theta_l).
    """
    s, th, M = layer_params(seed, layer)
    uv = scene.uv.astype(np.float64) @ M.T
    d = scene.duv.astype(np.float64)
    dx = d[..., 0:2] @ M.T
    dy = d[..., 2:4] @ M.T
    duv = np.concatenate([dx, dy], -1)
    return uv.astype(np.float32), duv.astype(np.float32), s, th


def head_on_quad_uv(tile_w, tile_h, magnification, angle_rad, offset, tex_w=4096):
    """uv of one tile of a head-on quad rotated in the image plane.

    The texel-space position of pixel centre (x+0.5, y+0.5) is
    R(angle) * (x+0.5, y+0.5) / magnification + offset; returned as float32
    uv (texel position / tex_w) with zero derivatives (magnifying).  This is
    the first scene of supplement S3 (head-on rotated quad), restricted to
    one tile.
    """
    ys, xs = np.mgrid[0:tile_h, 0:tile_w].astype(np.float64)
    c, s = math.cos(angle_rad), math.sin(angle_rad)
    px = xs + 0.5
    py = ys + 0.5
    tx = (c * px - s * py) / magnification + offset[0]
    ty = (s * px + c * py) / magnification + offset[1]
    uv = np.stack([tx / tex_w, ty / tex_w], -1).astype(np.float32)
    duv = np.zeros(uv.shape[:-1] + (4,), np.float32)
    return uv, duv


def lowmag_quads_scene(n_tiles=600, seed=21, tex_w=64, mag=(1.0, 1.3)):
    """A row of n_tiles 8x8 tiles, each a head-on quad at magnification drawn
    from ``mag`` with a random rotation and offset (zero derivatives).  Near
    magnification 1 an 8x8 tile needs more distinct texels than it has
    lanes, so waves with one evaluation per lane fail and take the fallback.
    Returns (uv [8][8 n][2], duv [8][8 n][4]) float32."""
    rng = np.random.default_rng(seed)
    mags = rng.uniform(mag[0], mag[1], n_tiles)
    angs = rng.uniform(0, math.pi / 2, n_tiles)
    offs = rng.uniform(0, tex_w, (n_tiles, 2))
    uv = np.zeros((8, 8 * n_tiles, 2), np.float32)
    for i in range(n_tiles):
        u, _ = head_on_quad_uv(8, 8, mags[i], angs[i], offs[i], tex_w=tex_w)
        uv[:, 8 * i:8 * i + 8] = u
    return uv, np.zeros(uv.shape[:2] + (4,), np.float32)


# ---------------------------------------------------------------------------
# decoder parameters
# ---------------------------------------------------------------------------

def decoder_layout(l0: int, l1: int, hidden: int, channels: int = 8):
    """Offsets of the flat decoder parameter vector.

    Order: latent level 0 [l0][l0][C], latent level 1 [l1][l1][C],
    W1 [2C][H], b1 [H], W2 [H][H], b2 [H], W3 [H][4], b3 [4]; weights are
    stored input-major (y_o = b_o + sum_i x_i W[i][o]).
    """
    sizes = [("lat0", l0 * l0 * channels), ("lat1", l1 * l1 * channels),
             ("W1", 2 * channels * hidden), ("b1", hidden),
             ("W2", hidden * hidden), ("b2", hidden),
             ("W3", hidden * 4), ("b3", 4)]
    off = {}
    o = 0
    for name, n in sizes:
        off[name] = (o, n)
        o += n
    off["total"] = (0, o)
    return off


def decoder_init(l0: int, l1: int, hidden: int, seed: int, channels: int = 8,
                 latent_range: float = 1e-2, out_bias: float = 0.5) -> np.ndarray:
    """Seeded initial parameters (float32 flat vector, layout of decoder_layout).

    Latents ~ U(-latent_range, latent_range); weights He-uniform
    (U(-sqrt(6/fan_in), +sqrt(6/fan_in))); hidden biases 0; output bias
    ``out_bias`` (the mean of a texture in [0, 1]).
    """
    lay = decoder_layout(l0, l1, hidden, channels)
    rng = np.random.default_rng(np.random.SeedSequence([0xDEC, seed]))
    p = np.zeros(lay["total"][1], dtype=np.float64)

    def put(name, vals):
        o, n = lay[name]
        p[o:o + n] = vals

    put("lat0", rng.uniform(-latent_range, latent_range, lay["lat0"][1]))
    put("lat1", rng.uniform(-latent_range, latent_range, lay["lat1"][1]))
    for name, fan_in in (("W1", 2 * channels), ("W2", hidden), ("W3", hidden)):
        lim = math.sqrt(6.0 / fan_in)
        put(name, rng.uniform(-lim, lim, lay[name][1]))
    put("b3", np.full(4, out_bias))
    return p.astype(np.float32)
