"""Seeded input generators (numpy PCG64) for the five workloads.

Every generator returns plain numpy arrays.  Complex samples are complex64
(the token type of the DPD channels), control tokens are int32 branch counts,
frames are uint8.  Nothing here computes an actor's output.

Workloads (sizes are the defaults; tests pass smaller ones):

* ``dpd_chain``     one DPD actor chain: 16384 i.i.d. complex Gaussian
  samples of unit RMS, 64 firings of 256 samples, control uniform in 1..5,
  8 taps, a unit linear tap, 4 zero delay tokens on the input channel.
* ``dpd_scale``     2**24 samples of an OFDM-like signal (complex Gaussian,
  band-limited to 80 % of the band, one clip at 10 dB above RMS), firings of
  4096 samples, control uniform in 1..10, 16 taps.
* ``motion``        300 grayscale 1920x1080 frames: static random texture,
  Gaussian noise sigma 3, 0..8 moving textured rectangles.
* ``dpd_instances`` 1024 independent DPD instances with lognormal lengths in
  [1024, 262144] (multiples of 1024), per-instance branch count in 1..10.
* ``adaptation``    64 streams x 65536 samples at RMS 0.25, a 7th-order
  4-tap memory-polynomial PA with random coefficients, DPD at identity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "DPDWorkload", "MotionWorkload", "InstancesWorkload", "AdaptWorkload",
    "complex_gaussian", "ofdm_like", "dpd_coeffs", "dpd_chain", "dpd_scale",
    "dpd_random", "motion", "paper_motion", "dpd_instances", "adaptation", "pa_coeffs",
    "papr_db",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def complex_gaussian(rng: np.random.Generator, n, rms: float = 1.0) -> np.ndarray:
    """i.i.d. circular complex Gaussian, Re and Im ~ N(0, rms^2/2), complex64."""
    shape = (n,) if np.isscalar(n) else tuple(n)
    s = rms / math.sqrt(2.0)
    re = rng.standard_normal(shape) * s
    im = rng.standard_normal(shape) * s
    return (re + 1j * im).astype(np.complex64)


def ofdm_like(rng: np.random.Generator, n: int, keep_frac: float = 0.8,
              clip_db: float = 10.0) -> np.ndarray:
    """OFDM-like stand-in: white CN(0,1) -> FFT -> zero bins with |f| > keep/2
    (central ``keep_frac`` of the band kept) -> IFFT -> unit RMS -> one
    phase-preserving amplitude clip at ``clip_db`` above RMS -> unit RMS."""
    w = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    f = np.fft.fftfreq(n)                      # cycles/sample in [-0.5, 0.5)
    spec = np.fft.fft(w)
    spec[np.abs(f) > keep_frac / 2.0] = 0.0
    s = np.fft.ifft(spec)
    s /= np.sqrt(np.mean(np.abs(s) ** 2))
    lim = 10.0 ** (clip_db / 20.0)
    mag = np.abs(s)
    over = mag > lim
    s[over] *= lim / mag[over]
    s /= np.sqrt(np.mean(np.abs(s) ** 2))
    return s.astype(np.complex64)


def papr_db(x: np.ndarray) -> float:
    p = np.abs(x.astype(np.complex128)) ** 2
    return float(10.0 * np.log10(p.max() / p.mean()))


def dpd_coeffs(rng: np.random.Generator, n_branches: int, n_taps: int,
               sigma: float = 0.1, factorial_scale: bool = True,
               unit_linear_tap: bool = True) -> np.ndarray:
    """Complex64 coefficients [n_branches][n_taps], Re and Im i.i.d.
    N(0, sigma^2).  Branch b (order 2b+1) is scaled by 1/sqrt((2b+1)!) when
    ``factorial_scale`` so that every branch contributes comparably for a
    unit-power Gaussian input; h[0][0] is then set to 1 (unit linear tap)."""
    h = (rng.standard_normal((n_branches, n_taps)) * sigma
         + 1j * rng.standard_normal((n_branches, n_taps)) * sigma)
    if factorial_scale:
        for b in range(1, n_branches):
            h[b] /= math.sqrt(math.factorial(2 * b + 1))
    if unit_linear_tap:
        h[0, 0] = 1.0
    return h.astype(np.complex64)


@dataclass
class DPDWorkload:
    x: np.ndarray            # complex64 [n_samples] pushed on the input channel
    ctrl: np.ndarray         # int32 [n_firings] control tokens (active branches)
    h: np.ndarray            # complex64 [n_branches_max][n_taps]
    r: int                   # samples per firing
    n_delay: int             # zero delay tokens on the input channel
    n_branches_max: int
    n_taps: int
    name: str = ""
    notes: dict = field(default_factory=dict)

    @property
    def n_firings(self) -> int:
        return int(self.ctrl.shape[0])


def dpd_chain(seed: int = 1, n_firings: int = 64, r: int = 256,
              n_branches_max: int = 5, n_taps: int = 8, n_delay: int = 4) -> DPDWorkload:
    """One DPD chain: i.i.d. unit-RMS complex Gaussian input, control uniform
    in 1..n_branches_max, coefficients N(0, 0.1^2) with a unit linear tap."""
    rng = _rng(seed)
    x = complex_gaussian(rng, n_firings * r)
    ctrl = rng.integers(1, n_branches_max + 1, size=n_firings).astype(np.int32)
    h = dpd_coeffs(rng, n_branches_max, n_taps, factorial_scale=False)
    return DPDWorkload(x, ctrl, h, r, n_delay, n_branches_max, n_taps,
                       name=f"dpd_chain_{n_firings}x{r}_B{n_branches_max}_M{n_taps}_d{n_delay}")


def dpd_scale(seed: int = 2, n_samples: int = 1 << 24, r: int = 4096,
              n_branches_max: int = 10, n_taps: int = 16) -> DPDWorkload:
    """DPD at scale: OFDM-like input, control uniform in 1..10, factorial-
    scaled coefficients, no delay tokens."""
    rng = _rng(seed)
    x = ofdm_like(rng, n_samples)
    n_firings = n_samples // r
    ctrl = rng.integers(1, n_branches_max + 1, size=n_firings).astype(np.int32)
    h = dpd_coeffs(rng, n_branches_max, n_taps, factorial_scale=True)
    return DPDWorkload(x, ctrl, h, r, 0, n_branches_max, n_taps,
                       name=f"dpd_scale_{n_samples}_r{r}_B{n_branches_max}_M{n_taps}",
                       notes={"papr_db": papr_db(x)})


def dpd_random(seed: int, n_firings: int, r: int, n_branches_max: int, n_taps: int,
               n_delay: int = 0, ctrl_low: int = 0, ctrl: np.ndarray | None = None,
               rms: float = 1.0, factorial_scale: bool = True) -> DPDWorkload:
    """Small parameterised DPD case for parity tests (any r, d, control range,
    including 0 = no active branch)."""
    rng = _rng(seed)
    x = complex_gaussian(rng, n_firings * r, rms=rms)
    if ctrl is None:
        ctrl = rng.integers(ctrl_low, n_branches_max + 1, size=n_firings)
    ctrl = np.asarray(ctrl, dtype=np.int32)
    h = dpd_coeffs(rng, n_branches_max, n_taps, factorial_scale=factorial_scale)
    return DPDWorkload(x, ctrl, h, r, n_delay, n_branches_max, n_taps,
                       name=f"dpd_random_s{seed}_{n_firings}x{r}_B{n_branches_max}_M{n_taps}_d{n_delay}")


# ---------------------------------------------------------------- motion

@dataclass
class MotionWorkload:
    frames: np.ndarray       # uint8 [n_frames][height][width]
    width: int
    height: int
    threshold: int = 25      # changed iff |cur - prev| > threshold
    min_changed_permille: int = 1   # emit iff 1000*count >= permille*W*H
    name: str = ""
    notes: dict = field(default_factory=dict)


def motion(seed: int = 3, n_frames: int = 300, width: int = 1920, height: int = 1080,
           n_tracks: int = 8, noise_sigma: float = 3.0, segment: int = 20,
           rect_min: int = 32, rect_max: int = 256, vmax: int = 12) -> MotionWorkload:
    """Static uniform-u8 background texture + moving textured rectangles +
    N(0, sigma^2) noise, rounded half-to-even and clipped to [0, 255].

    Rectangle tracks: size U[rect_min, rect_max]^2 (clamped to the frame),
    own uniform-u8 texture, integer velocity U[-vmax, vmax]^2 without (0, 0),
    reflecting at the frame edges.  The number of visible tracks is drawn
    uniformly in 0..n_tracks once per ``segment`` frames (the first k tracks
    are the visible ones)."""
    rng = _rng(seed)
    bg = rng.integers(0, 256, size=(height, width), dtype=np.int64).astype(np.uint8)
    tracks = []
    for _ in range(n_tracks):
        rh = int(min(rng.integers(rect_min, rect_max + 1), height))
        rw = int(min(rng.integers(rect_min, rect_max + 1), width))
        tex = rng.integers(0, 256, size=(rh, rw), dtype=np.int64).astype(np.uint8)
        y = int(rng.integers(0, height - rh + 1))
        x = int(rng.integers(0, width - rw + 1))
        while True:
            vy, vx = (int(v) for v in rng.integers(-vmax, vmax + 1, size=2))
            if (vy, vx) != (0, 0):
                break
        tracks.append([y, x, vy, vx, rh, rw, tex])
    n_seg = (n_frames + segment - 1) // segment
    visible = rng.integers(0, n_tracks + 1, size=n_seg)
    frames = np.empty((n_frames, height, width), dtype=np.uint8)
    for t in range(n_frames):
        img = bg.astype(np.float64)
        k = int(visible[t // segment])
        for tr in tracks[:k]:
            y, x, _, _, rh, rw, tex = tr
            img[y:y + rh, x:x + rw] = tex
        img += rng.standard_normal((height, width)) * noise_sigma
        frames[t] = np.clip(np.rint(img), 0, 255).astype(np.uint8)
        for tr in tracks:           # every track moves, visible or not
            y, x, vy, vx, rh, rw, _ = tr
            ny, nx = y + vy, x + vx
            if ny < 0 or ny > height - rh:
                vy = -vy
                ny = y + vy
            if nx < 0 or nx > width - rw:
                vx = -vx
                nx = x + vx
            tr[0] = min(max(ny, 0), height - rh)
            tr[1] = min(max(nx, 0), width - rw)
            tr[2], tr[3] = vy, vx
    return MotionWorkload(frames, width, height,
                          name=f"motion_{n_frames}x{width}x{height}",
                          notes={"visible_per_segment": visible.tolist()})


def paper_motion(seed: int = 6, n_frames: int = 64, width: int = 320, height: int = 240) -> MotionWorkload:
    """Frames for the paper's motion-detection pipeline: 8-bit grayscale at
    the paper's 320x240 (one 76,800-byte token per frame), the same recipe as
    ``motion`` with rectangles scaled to the frame (16..80 pixels a side,
    speed up to 6 pixels per frame, noise sigma 3)."""
    w = motion(seed=seed, n_frames=n_frames, width=width, height=height, n_tracks=8, noise_sigma=3.0,
               segment=20, rect_min=min(16, width, height), rect_max=min(80, width, height), vmax=6)
    w.name = f"paper_motion_{n_frames}x{width}x{height}"
    return w


# ---------------------------------------------------------------- batched instances

@dataclass
class InstancesWorkload:
    lengths: np.ndarray      # int64 [n_instances], multiples of r
    n_branches: np.ndarray   # int32 [n_instances], constant control per instance
    x: list                  # list of complex64 arrays
    h: np.ndarray            # complex64 [n_instances][n_branches_max][n_taps]
    r: int
    n_branches_max: int
    n_taps: int
    name: str = ""

    def ctrl(self, i: int) -> np.ndarray:
        return np.full(int(self.lengths[i]) // self.r, int(self.n_branches[i]), np.int32)


def dpd_instances(seed: int = 4, n_instances: int = 1024, r: int = 1024,
                  len_min: int = 1024, len_max: int = 262144, median: int = 16384,
                  sigma: float = 1.0, n_branches_max: int = 10, n_taps: int = 16,
                  with_signals: bool = True) -> InstancesWorkload:
    """Lengths L = clip(floor_r(exp(N(ln median, sigma))), len_min, len_max),
    branch count uniform in 1..n_branches_max per instance, per-instance
    factorial-scaled coefficients, unit-RMS complex Gaussian input."""
    rng = _rng(seed)
    raw = np.exp(rng.normal(math.log(median), sigma, size=n_instances))
    lengths = (np.floor(raw / r) * r).astype(np.int64)
    lengths = np.clip(lengths, len_min, len_max)
    nb = rng.integers(1, n_branches_max + 1, size=n_instances).astype(np.int32)
    h = np.stack([dpd_coeffs(rng, n_branches_max, n_taps) for _ in range(n_instances)])
    xs = [complex_gaussian(rng, int(L)) for L in lengths] if with_signals else []
    return InstancesWorkload(lengths, nb, xs, h, r, n_branches_max, n_taps,
                             name=f"dpd_instances_{n_instances}_r{r}")


# ---------------------------------------------------------------- adaptation

@dataclass
class AdaptWorkload:
    x: np.ndarray            # complex64 [n_streams][length]
    h0: np.ndarray           # complex64 [n_branches][n_taps] initial DPD (identity)
    a: np.ndarray            # complex64 [n_pa_branches][n_pa_taps], orders 1,3,5,7
    name: str = ""


def pa_coeffs(rng: np.random.Generator, n_branches: int = 4, n_taps: int = 4,
              sigma: float = 0.05) -> np.ndarray:
    """PA memory polynomial coefficients a[k][q] (order 2k+1, delay q):
    a[0][0] = 1, all others Re, Im ~ N(0, sigma^2)."""
    a = (rng.standard_normal((n_branches, n_taps)) * sigma
         + 1j * rng.standard_normal((n_branches, n_taps)) * sigma)
    a[0, 0] = 1.0
    return a.astype(np.complex64)


def adaptation(seed: int = 5, n_streams: int = 64, length: int = 65536,
               n_branches: int = 10, n_taps: int = 16, rms: float = 0.25) -> AdaptWorkload:
    rng = _rng(seed)
    x = complex_gaussian(rng, (n_streams, length), rms=rms)
    a = pa_coeffs(rng)
    h0 = np.zeros((n_branches, n_taps), np.complex64)
    h0[0, 0] = 1.0
    return AdaptWorkload(x, h0, a, name=f"adaptation_{n_streams}x{length}_B{n_branches}_M{n_taps}")
