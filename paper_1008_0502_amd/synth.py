"""Seeded synthetic video clips (uint8 RGB frames plus ground-truth object masks).

The paper evaluates on ten private clips (5-10 s at 12 fps, Section "Conditions"
of the experiments) that are not available; these generators stand in for them.
This module holds none of the saliency/prior arithmetic: it only draws pixels.
It is the one module that both the CPU oracle tests and the HIP path consume.

Recipe (all geometry in float64, pixel values rounded with floor(v + 0.5)):

* ellipse: axis-aligned, centre (cx, cy), semi-axes (a, b); a pixel (x, y)
  (integer indices = pixel centres) is inside iff ((x-cx)/a)^2 + ((y-cy)/b)^2 <= 1;
* texture: colour * (0.75 + 0.25*cos(2*pi*(x - cx)/4)), attached to the object;
* motion: start centre uniform with the bounding box inside the frame; velocity
  either speed*(cos phi, sin phi) with phi ~ U[0, 2 pi) or uniform in a disc;
  a velocity component is reflected when the box would leave the frame;
* colours: "saturated" picks one of R, G, B, C, M, Y at 255; "hsv" draws
  HSV(h ~ U[0,1), s = 1, v = 1);
* background: static per clip, either uniform noise U{0..255} per channel or
  three independent Perlin gradient-noise fields (4 octaves, base cell 64 px,
  persistence 0.5), each min-max mapped to [0, 255].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional, Sequence, Tuple

import numpy as np

_SATURATED = np.array(
    [[255, 0, 0], [0, 255, 0], [0, 0, 255], [0, 255, 255], [255, 0, 255], [255, 255, 0]],
    dtype=np.float64,
)


def _round_u8(v: np.ndarray) -> np.ndarray:
    return np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8)


def _hsv_full(h: float) -> np.ndarray:
    """HSV(h, 1, 1) -> RGB in [0, 255] (float64)."""
    h6 = (h % 1.0) * 6.0
    i = int(math.floor(h6)) % 6
    f = h6 - math.floor(h6)
    q, t = 1.0 - f, f
    table = [(1, t, 0), (q, 1, 0), (0, 1, t), (0, q, 1), (t, 0, 1), (1, 0, q)]
    return np.array(table[i], dtype=np.float64) * 255.0


def _fade(t: np.ndarray) -> np.ndarray:
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def perlin_field(rng: np.random.Generator, H: int, W: int, octaves: int = 4,
                 base_cell: float = 64.0, persistence: float = 0.5) -> np.ndarray:
    """One 2-D gradient-noise field (Perlin's construction: random unit gradients on
    a lattice, quintic fade, bilinear blend of the corner dot products), summed over
    octaves with halving cell size and amplitude `persistence**o`."""
    ys = np.arange(H, dtype=np.float64)
    xs = np.arange(W, dtype=np.float64)
    out = np.zeros((H, W), dtype=np.float64)
    for o in range(octaves):
        cell = base_cell / (2 ** o)
        gy = int(math.ceil(H / cell)) + 2
        gx = int(math.ceil(W / cell)) + 2
        ang = rng.uniform(0.0, 2.0 * math.pi, size=(gy, gx))
        gxv, gyv = np.cos(ang), np.sin(ang)
        v = ys / cell
        u = xs / cell
        i0 = np.floor(v).astype(np.int64)
        j0 = np.floor(u).astype(np.int64)
        fv = (v - i0)[:, None]
        fu = (u - j0)[None, :]
        I0, J0 = i0[:, None], j0[None, :]

        def corner(di: int, dj: int) -> np.ndarray:
            gx_ = gxv[I0 + di, J0 + dj]
            gy_ = gyv[I0 + di, J0 + dj]
            return gx_ * (fu - dj) + gy_ * (fv - di)

        su, sv = _fade(fu), _fade(fv)
        top = corner(0, 0) * (1 - su) + corner(0, 1) * su
        bot = corner(1, 0) * (1 - su) + corner(1, 1) * su
        out += (persistence ** o) * (top * (1 - sv) + bot * sv)
    return out


@dataclasses.dataclass
class ClipSpec:
    """Parameters of one synthetic clip."""
    H: int
    W: int
    T: int
    background: str = "uniform"          # "uniform" | "perlin"
    n_objects: int = 1
    axes: Optional[Tuple[float, float]] = (15.0, 10.0)   # fixed (a, b); None -> random
    axes_range: Tuple[float, float] = (10.0, 40.0)
    speed: Optional[float] = 2.0          # fixed speed with random direction
    max_speed: float = 4.0                # used when speed is None (uniform in a disc)
    colours: str = "saturated"           # "saturated" | "hsv"
    seed: int = 0


@dataclasses.dataclass
class _Obj:
    cx: float
    cy: float
    a: float
    b: float
    vx: float
    vy: float
    colour: np.ndarray


class Clip:
    """A seeded clip; frames are rendered lazily so long clips need no storage."""

    def __init__(self, spec: ClipSpec):
        self.spec = spec
        rng = np.random.default_rng(spec.seed)
        H, W = spec.H, spec.W
        if spec.background == "uniform":
            self.background = rng.integers(0, 256, size=(H, W, 3), dtype=np.int64).astype(np.uint8)
        elif spec.background == "perlin":
            chans = []
            for _ in range(3):
                f = perlin_field(rng, H, W)
                lo, hi = f.min(), f.max()
                chans.append((f - lo) / (hi - lo) * 255.0 if hi > lo else np.zeros_like(f))
            self.background = _round_u8(np.stack(chans, axis=2))
        else:
            raise ValueError(f"unknown background {spec.background!r}")
        self.objects: List[_Obj] = []
        for _ in range(spec.n_objects):
            if spec.axes is not None:
                a, b = spec.axes
            else:
                a = rng.uniform(*spec.axes_range)
                b = rng.uniform(*spec.axes_range)
            a = min(a, (W - 1) / 2.0)
            b = min(b, (H - 1) / 2.0)
            cx = rng.uniform(a, W - 1 - a)
            cy = rng.uniform(b, H - 1 - b)
            if spec.speed is not None:
                phi = rng.uniform(0.0, 2.0 * math.pi)
                vx, vy = spec.speed * math.cos(phi), spec.speed * math.sin(phi)
            else:
                r = spec.max_speed * math.sqrt(rng.uniform(0.0, 1.0))
                phi = rng.uniform(0.0, 2.0 * math.pi)
                vx, vy = r * math.cos(phi), r * math.sin(phi)
            if spec.colours == "saturated":
                colour = _SATURATED[rng.integers(0, 6)]
            else:
                colour = _hsv_full(rng.uniform(0.0, 1.0))
            self.objects.append(_Obj(cx, cy, a, b, vx, vy, colour))
        self._state_t = 0
        self._positions = [(o.cx, o.cy, o.vx, o.vy) for o in self.objects]
        self._xs = np.arange(W, dtype=np.float64)[None, :]
        self._ys = np.arange(H, dtype=np.float64)[:, None]

    # -- motion ---------------------------------------------------------------
    def _advance(self) -> None:
        W, H = self.spec.W, self.spec.H
        new = []
        for o, (cx, cy, vx, vy) in zip(self.objects, self._positions):
            nx = cx + vx
            if nx - o.a < 0 or nx + o.a > W - 1:
                vx = -vx
                nx = cx + vx
            ny = cy + vy
            if ny - o.b < 0 or ny + o.b > H - 1:
                vy = -vy
                ny = cy + vy
            new.append((nx, ny, vx, vy))
        self._positions = new

    def _seek(self, t: int) -> None:
        if t < self._state_t:
            self._positions = [(o.cx, o.cy, o.vx, o.vy) for o in self.objects]
            self._state_t = 0
        while self._state_t < t:
            self._advance()
            self._state_t += 1

    # -- rendering ------------------------------------------------------------
    def frame(self, t: int) -> Tuple[np.ndarray, np.ndarray]:
        """(rgb uint8 [H][W][3], mask uint8 [H][W]) of frame t."""
        self._seek(t)
        H, W = self.spec.H, self.spec.W
        img = self.background.copy()
        mask = np.zeros((H, W), dtype=np.uint8)
        for o, (cx, cy, _, _) in zip(self.objects, self._positions):
            # only pixels of the bounding box can be inside; later objects cover earlier ones
            x0, x1 = max(0, int(math.floor(cx - o.a))), min(W, int(math.ceil(cx + o.a)) + 1)
            y0, y1 = max(0, int(math.floor(cy - o.b))), min(H, int(math.ceil(cy + o.b)) + 1)
            if x0 >= x1 or y0 >= y1:
                continue
            xs, ys = self._xs[:, x0:x1], self._ys[y0:y1, :]
            inside = ((xs - cx) / o.a) ** 2 + ((ys - cy) / o.b) ** 2 <= 1.0
            tex = 0.75 + 0.25 * np.cos(2.0 * math.pi * (xs - cx) / 4.0)
            val = _round_u8(o.colour[None, None, :] * np.broadcast_to(tex, inside.shape)[:, :, None])
            win = img[y0:y1, x0:x1]
            win[inside] = val[inside]
            mask[y0:y1, x0:x1] |= inside.astype(np.uint8)
        return img, mask

    def frames(self, t0: int = 0, t1: Optional[int] = None) -> Iterator[Tuple[np.ndarray, np.ndarray]]:
        t1 = self.spec.T if t1 is None else t1
        for t in range(t0, t1):
            yield self.frame(t)

    def stack(self, t0: int = 0, t1: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
        """All frames in [t0, t1) as arrays [T][H][W][3] and [T][H][W]."""
        fr = list(self.frames(t0, t1))
        return np.stack([f for f, _ in fr]), np.stack([m for _, m in fr])


# -- the named workloads -------------------------------------------------------
def single_ellipse_spec(H: int = 120, W: int = 160, T: int = 30, seed: int = 0) -> ClipSpec:
    """Uniform-noise background, one saturated 15x10 ellipse, 2 px/frame."""
    return ClipSpec(H=H, W=W, T=T, background="uniform", n_objects=1, axes=(15.0, 10.0),
                    speed=2.0, colours="saturated", seed=seed)


def three_ellipse_spec(H: int = 240, W: int = 320, T: int = 300, seed: int = 1) -> ClipSpec:
    """Perlin background, three random-colour ellipses, radii 10-40, speed <= 4."""
    return ClipSpec(H=H, W=W, T=T, background="perlin", n_objects=3, axes=None,
                    axes_range=(10.0, 40.0), speed=None, max_speed=4.0, colours="hsv", seed=seed)


def five_ellipse_spec(H: int = 1080, W: int = 1920, T: int = 1000, seed: int = 5) -> ClipSpec:
    """Perlin background, five random-colour ellipses, speed <= 8; radii scaled
    from the 240-row family by H/240."""
    s = H / 240.0
    return ClipSpec(H=H, W=W, T=T, background="perlin", n_objects=5, axes=None,
                    axes_range=(10.0 * s, 40.0 * s), speed=None, max_speed=8.0, colours="hsv",
                    seed=seed)


def mixed_batch_specs(T: int = 60, per_size: int = 16, base_seed: int = 1000,
                      sizes: Sequence[Tuple[int, int]] = ((120, 160), (240, 320), (480, 640), (720, 1280))
                      ) -> List[ClipSpec]:
    """Many streams of uneven resolution, single-ellipse generator, seeds base_seed + i."""
    specs = []
    i = 0
    for (H, W) in sizes:
        for _ in range(per_size):
            specs.append(single_ellipse_spec(H=H, W=W, T=T, seed=base_seed + i))
            i += 1
    return specs


def constant_frame(H: int, W: int, rgb: Sequence[int]) -> np.ndarray:
    f = np.empty((H, W, 3), dtype=np.uint8)
    f[...] = np.asarray(rgb, dtype=np.uint8)
    return f


def random_frames(rng: np.random.Generator, T: int, H: int, W: int) -> np.ndarray:
    """Uniform-noise frames (every pixel independent), for tiny brute-force cases."""
    return rng.integers(0, 256, size=(T, H, W, 3), dtype=np.int64).astype(np.uint8)
