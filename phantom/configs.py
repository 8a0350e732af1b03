"""Workload descriptions: probe, transmit sequence, pixel grid and phantom.

Geometry conventions (readings of the paper, which names only speed of sound,
aperture size and sampling frequency as acquisition metadata, Sec. II-A):

* linear array on z = 0, element e at x_e = (e - (N-1)/2) * pitch unless an
  explicit element list is given;
* z is depth (positive into the medium); pixel (iz, ix) sits at
  (x0 + ix*dx, z0 + iz*dz); grid end points are inclusive;
* lateral extent of every grid is the element span [x_0, x_{N-1}];
* STAI: transmit t fires element ``tx_elem[t]`` (default t);
* PWI: transmit k is a plane wave steered by angle theta_k (> 0 towards +x),
  time zero when the first element fires (``tref="first"``) or when the
  wavefront crosses the array centre (``tref="centre"``);
* receive channel j is element ``rx_elem[j]`` (default j);
* the RF record starts at t0 = 0 and sample s is taken at t0 + s/fs.

The five named workloads follow the evaluation setups of the build: a small
STAI case, a full-size STAI wire phantom, a PWI cyst phantom, an 8-frame PWI
batch, and a served mixed stream.  The paper's own shapes (STAI 128 x 64 x
2048, PWI 11 x 192 x 2048, Sec. III) are available as ``paper_stai`` and
``paper_pwi`` for context timing.
"""

from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

MM = 1e-3


@dataclass(frozen=True)
class Workload:
    name: str
    mode: str  # "stai" | "pwi"
    n_elem: int
    pitch: float  # m
    fc: float  # Hz, pulse centre frequency (generator only)
    fs: float  # Hz
    c: float  # m/s
    n_tx: int
    n_ch: int
    n_s: int
    nz: int
    nx: int
    z_min: float  # m
    z_max: float  # m
    n_frames: int = 1
    t0: float = 0.0
    f_number: float = 0.0
    dr_db: float = 60.0
    tx_elem: Optional[Tuple[int, ...]] = None  # STAI
    angles_deg: Optional[Tuple[float, ...]] = None  # PWI
    tref: str = "first"
    rx_elem: Optional[Tuple[int, ...]] = None
    x_min: Optional[float] = None  # default: first element
    x_max: Optional[float] = None  # default: last element
    phantom: str = "points"
    phantom_args: dict = field(default_factory=dict)
    snr_db: Optional[float] = None
    seed: int = 0

    def __post_init__(self):
        # the per-transmit and per-channel lists must describe every transmit
        # and channel: the library reads n_tx angles (or elements) and n_ch
        # channel elements
        if self.mode == "pwi" and (self.angles_deg is None or len(self.angles_deg) != self.n_tx):
            raise ValueError(f"{self.name}: {self.n_tx} plane waves need as many angles_deg")
        if self.tx_elem is not None and len(self.tx_elem) != self.n_tx:
            raise ValueError(f"{self.name}: tx_elem has {len(self.tx_elem)} entries, "
                             f"n_tx={self.n_tx}")
        if self.rx_elem is not None and len(self.rx_elem) != self.n_ch:
            raise ValueError(f"{self.name}: rx_elem has {len(self.rx_elem)} entries, "
                             f"n_ch={self.n_ch}")

    # ----- derived geometry -------------------------------------------------
    def elem_x(self) -> list:
        """Element lateral positions (m), centred uniform linear array."""
        return [(e - (self.n_elem - 1) / 2.0) * self.pitch for e in range(self.n_elem)]

    def grid(self) -> dict:
        xs = self.elem_x()
        xa = xs[0] if self.x_min is None else self.x_min
        xb = xs[-1] if self.x_max is None else self.x_max
        dz = (self.z_max - self.z_min) / (self.nz - 1) if self.nz > 1 else 0.0
        dx = (xb - xa) / (self.nx - 1) if self.nx > 1 else 0.0
        return dict(nz=self.nz, nx=self.nx, z0=self.z_min, dz=dz, x0=xa, dx=dx)

    def tx_elements(self) -> list:
        if self.tx_elem is not None:
            return list(self.tx_elem)
        return list(range(self.n_tx))

    def rx_elements(self) -> list:
        if self.rx_elem is not None:
            return list(self.rx_elem)
        return list(range(self.n_ch))

    def angles_rad(self) -> list:
        return [math.radians(a) for a in self.angles_deg]

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    # contributions = pixels x transmits x channels (one interpolate-and-add)
    @property
    def nominal_contributions(self) -> int:
        return self.n_frames * self.nz * self.nx * self.n_tx * self.n_ch


def _linspace(a: float, b: float, n: int) -> Tuple[float, ...]:
    if n == 1:
        return (0.5 * (a + b),)
    return tuple(a + (b - a) * i / (n - 1) for i in range(n))


def _stai_small() -> Workload:
    # 32 elements, 32 single-element transmits x 32 channels x 1024 samples,
    # five point scatterers, 20 dB white noise; 128 x 128 grid over 0-30 mm.
    return Workload(
        name="stai_small", mode="stai", n_elem=32, pitch=0.3 * MM, fc=5e6, fs=50e6,
        c=1540.0, n_tx=32, n_ch=32, n_s=1024, nz=128, nx=128, z_min=0.0, z_max=30 * MM,
        phantom="points_on_pixels",
        phantom_args=dict(pixels=((21, 64), (34, 32), (34, 96), (47, 64), (59, 20))),
        snr_db=20.0, seed=1,
    )


def _stai_full() -> Workload:
    # 128 x 128 x 2048, wire lattice + 10k weak speckle, 1024 x 256 grid over
    # 5-50 mm, f/1.5 receive aperture.
    return Workload(
        name="stai_full", mode="stai", n_elem=128, pitch=0.3 * MM, fc=5.5e6, fs=50e6,
        c=1540.0, n_tx=128, n_ch=128, n_s=2048, nz=1024, nx=256, z_min=5 * MM,
        z_max=50 * MM, f_number=1.5, phantom="wires_speckle",
        phantom_args=dict(
            wires_x_mm=(-7.5, -2.5, 2.5, 7.5), wires_z_mm=(10, 15, 20, 25, 30),
            n_speckle=10_000, speckle_sigma=0.05, z_range_mm=(5.0, 50.0)),
        seed=2,
    )


def _pwi() -> Workload:
    # 64 plane waves over -16..+16 deg x 128 channels x 2048 samples, 200k
    # Rayleigh speckle with three 4 mm anechoic cysts, 1024 x 512 grid over
    # 5-30 mm, coherent compounding.
    return Workload(
        name="pwi", mode="pwi", n_elem=128, pitch=0.3 * MM, fc=5.5e6, fs=50e6, c=1540.0,
        n_tx=64, n_ch=128, n_s=2048, nz=1024, nx=512, z_min=5 * MM, z_max=30 * MM,
        angles_deg=_linspace(-16.0, 16.0, 64), phantom="cysts",
        phantom_args=dict(n_speckle=200_000, z_range_mm=(5.0, 30.0), cyst_radius_mm=2.0,
                          cysts_mm=((-10.0, 12.0), (0.0, 18.0), (10.0, 24.0))),
        seed=3,
    )


def _pwi_batch() -> Workload:
    return _pwi().with_(name="pwi_batch8", n_frames=8, seed=4)


def _paper_stai() -> Workload:
    # Paper shape (Sec. III): 128 acquisitions x 64 channels x 2048 samples,
    # output 2048 x 128, clipped to 30 dB.  Receive channels map to the 64
    # elements centred on the transmit element in the paper's scanner; here
    # (fixed channel map across transmits) channels are elements 32..95.
    return Workload(
        name="paper_stai", mode="stai", n_elem=128, pitch=0.3 * MM, fc=5.5e6, fs=50e6,
        c=1540.0, n_tx=128, n_ch=64, n_s=2048, nz=2048, nx=128, z_min=5 * MM,
        z_max=30 * MM, rx_elem=tuple(range(32, 96)), dr_db=30.0,
        phantom="cysts", phantom_args=dict(n_speckle=20_000, z_range_mm=(5.0, 30.0),
                                           cyst_radius_mm=2.0, cysts_mm=((0.0, 18.0),)),
        seed=5,
    )


def _paper_pwi() -> Workload:
    return Workload(
        name="paper_pwi", mode="pwi", n_elem=192, pitch=0.2 * MM, fc=5.5e6, fs=50e6,
        c=1540.0, n_tx=11, n_ch=192, n_s=2048, nz=512, nx=128, z_min=5 * MM,
        z_max=30 * MM, angles_deg=_linspace(-16.0, 16.0, 11), dr_db=30.0,
        phantom="cysts", phantom_args=dict(n_speckle=20_000, z_range_mm=(5.0, 30.0),
                                           cyst_radius_mm=2.0, cysts_mm=((0.0, 18.0),)),
        seed=6,
    )


def tiny_stai(**kw) -> Workload:
    """Tiny STAI case for brute-force checks (N=4, T=4, S=64, 6 x 5 grid)."""
    w = Workload(
        name="tiny_stai", mode="stai", n_elem=4, pitch=0.3 * MM, fc=5e6, fs=50e6,
        c=1540.0, n_tx=4, n_ch=4, n_s=64, nz=6, nx=5, z_min=0.2 * MM, z_max=0.8 * MM,
        phantom="random", seed=11,
    )
    return w.with_(**kw) if kw else w


def tiny_pwi(**kw) -> Workload:
    """Tiny PWI case for brute-force checks (N=4, 3 angles, S=64, 6 x 5 grid)."""
    w = Workload(
        name="tiny_pwi", mode="pwi", n_elem=4, pitch=0.3 * MM, fc=5e6, fs=50e6,
        c=1540.0, n_tx=3, n_ch=4, n_s=64, nz=6, nx=5, z_min=0.2 * MM, z_max=0.8 * MM,
        angles_deg=(-12.0, 0.0, 9.0), phantom="random", seed=12,
    )
    return w.with_(**kw) if kw else w


WORKLOADS = {
    "stai_small": _stai_small,
    "stai_full": _stai_full,
    "pwi": _pwi,
    "pwi_batch8": _pwi_batch,
    "paper_stai": _paper_stai,
    "paper_pwi": _paper_pwi,
}


def get_workload(name: str, **overrides) -> Workload:
    w = WORKLOADS[name]()
    return w.with_(**overrides) if overrides else w


def subgrid(w: Workload, iz0: int, nz: int, ix0: int, nx: int) -> Workload:
    """The same acquisition imaged on a rectangular sub-window of its grid."""
    g = w.grid()
    z0 = g["z0"] + iz0 * g["dz"]
    x0 = g["x0"] + ix0 * g["dx"]
    return w.with_(nz=nz, nx=nx, z_min=z0, z_max=z0 + (nz - 1) * g["dz"],
                   x_min=x0, x_max=x0 + (nx - 1) * g["dx"])


def served_mix(seed: int = 7) -> Sequence[Workload]:
    """Shape classes of the served mixed stream: STAI or PWI, N in
    {64,128,192}, T in {16,32,64,128} (STAI: T <= N, evenly spaced transmit
    elements), S in {1024,2048,4096}, grids {256x128, 512x256, 1024x512}."""
    out = []
    for mode in ("stai", "pwi"):
        for n in (64, 128, 192):
            for t in (16, 32, 64, 128):
                if mode == "stai" and t > n:
                    continue
                for s in (1024, 2048, 4096):
                    for (nz, nx) in ((256, 128), (512, 256), (1024, 512)):
                        kw = dict(
                            name=f"{mode}_n{n}_t{t}_s{s}_{nz}x{nx}", mode=mode, n_elem=n,
                            pitch=0.3 * MM, fc=5.5e6, fs=50e6, c=1540.0, n_tx=t, n_ch=n,
                            n_s=s, nz=nz, nx=nx, z_min=5 * MM, z_max=30 * MM,
                            phantom="cysts",
                            phantom_args=dict(n_speckle=4000, z_range_mm=(5.0, 30.0),
                                              cyst_radius_mm=2.0, cysts_mm=((0.0, 18.0),)),
                            seed=seed)
                        if mode == "stai":
                            kw["tx_elem"] = tuple(int(round(i * (n - 1) / max(t - 1, 1)))
                                                  for i in range(t))
                        else:
                            kw["angles_deg"] = _linspace(-16.0, 16.0, t)
                        out.append(Workload(**kw))
    return out


def served_pool(n_classes: int = 16, seed: int = 7) -> Sequence[Workload]:
    """A seeded subset of the served-mix shape classes, each with its own
    seeded speckle + cyst phantom (4000 Rayleigh scatterers, one 4 mm
    anechoic cyst); the served stream draws its requests from one RF frame
    per class."""
    import random

    mix = list(served_mix(seed))
    rnd = random.Random(seed)
    picks = rnd.sample(range(len(mix)), n_classes)
    return [mix[i].with_(seed=seed * 1000 + k) for k, i in enumerate(sorted(picks))]


# qUS moment maps of the envelope: window 32 depth samples (about three pulse
# lengths on the 1024-row grids) x 8 columns, strides 8 x 2 (75 % overlap)
QUS_WINDOW = dict(wz=32, wx=8, sz=8, sx=2)
# FIR pre-filter: 31-tap Hamming band-pass over [0.5 fc, 1.5 fc]
FIR_TAPS = 31
