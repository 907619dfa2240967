"""Problem cards: every number that defines a synthetic workload, in SI units.

A card is plain data.  Lengths are metres, times seconds, speeds m/s,
densities kg/m^3, attenuation s/m (the unit the paper gives next to Eq. (3)),
frequencies Hz.  The three cards follow the three single-problem workloads of
the method's evaluation plan: a small plain case (64x64), a plain FP32 case
(256x256, 32 scan positions) and a large precision case (512x512, four layers).

The medium is a stack of planar layers under the array; the array sits on
z = 0, the top of layer 1 (Fig. 1); the last layer extends downward without end.
Transducer x positions are absolute.  Receiver positions are offsets from the
transmitter of the same scan position (the assembly moves as a unit).
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict
from typing import Optional, Tuple

MM = 1e-3
US = 1e-6
MHZ = 1e6


@dataclass(frozen=True)
class Medium:
    speed: Tuple[float, ...]          # c_l [m/s], layer 1 first
    thickness: Tuple[float, ...]      # eta of layers 1..L-1 [m]; layer L is unbounded
    atten: Tuple[float, ...]          # alpha_l [s/m]
    density: Tuple[float, ...]        # rho_l [kg/m^3]
    names: Tuple[str, ...] = ()

    @property
    def n_layers(self) -> int:
        return len(self.speed)


@dataclass(frozen=True)
class Grid:
    nx: int
    nz: int
    dx: float
    dz: float
    x0: float        # left edge of column 0 [m]
    z0: float = 0.0  # top edge of row 0 [m]


@dataclass(frozen=True)
class Array:
    tx_x: Tuple[float, ...]       # P transmitter (scan) positions [m]
    rx_offset: Tuple[float, ...]  # K receiver offsets from the transmitter [m]
    beta: int = 8                 # apodization power of Eq. (12)

    @property
    def n_scans(self) -> int:
        return len(self.tx_x)

    @property
    def n_rx(self) -> int:
        return len(self.rx_offset)


@dataclass(frozen=True)
class Acquisition:
    n_samples: int     # M
    fs: float          # sampling rate [Hz]; sample m is at t = m / fs after firing
    f_c: float         # pulse centre frequency [Hz]
    sigma_t: float     # pulse Gaussian width [s]
    t_win: float       # window length t_0 of Eq. (10) [s]
    oversample: int    # template oversampling factor Q
    storage: int = 0   # element type of traces in the sweeps: 0 FP32, 1 FP16, 2 BF16
    n_gamma: int = 16  # attenuation templates when some alpha_l > 0 (2..64)


@dataclass(frozen=True)
class Prior:
    p: float = 1.1       # Eq. (15) shape
    q: float = 2.0
    T: float = 0.01      # threshold of Eq. (15)
    sigma0: float = 5.0  # Eq. (16)
    m: float = 0.1       # depth modulation of Eq. (17)
    a: float = 1.0
    estimate_direct: bool = True


@dataclass(frozen=True)
class PhantomSpec:
    seed: int
    n_reflectors: int
    amp_lo: float
    amp_hi: float
    rows: Tuple[int, int]       # half-open row band for point reflectors
    cols: Tuple[int, int]       # half-open column band
    min_spacing: int            # Chebyshev distance between reflectors [voxels]
    interfaces: Tuple[Tuple[int, float], ...] = ()   # (row, reflectivity) full-width rows
    # debonding gap: (row, thick_lo, thick_hi [m], span_lo, span_hi [fraction of nx],
    #                 R_top, R_bottom, R_outside) -- R_outside replaces the interface
    #                 reflectivity of `row` outside the gap's lateral span.
    gap: Optional[Tuple[int, float, float, float, float, float, float, float]] = None


@dataclass(frozen=True)
class Card:
    name: str
    medium: Medium
    grid: Grid
    array: Array
    acq: Acquisition
    prior: Prior
    phantom: PhantomSpec
    snr_db: float
    noise_seed: int
    n_iter: int

    def to_dict(self):
        return asdict(self)

    @property
    def n_traces(self) -> int:
        return self.array.n_scans * self.array.n_rx

    @property
    def n_voxels(self) -> int:
        return self.grid.nx * self.grid.nz


# Reflectivities (Z2 - Z1)/(Z2 + Z1) of the phantom interfaces, with
# Z = density * speed for water 1000*1480, steel 7850*5900, cement 1900*3000,
# rock 2600*4500 (values rounded to four digits).
R_WATER_STEEL = 0.9381
R_STEEL_CEMENT = -0.7808
R_STEEL_WATER = -0.9381
R_WATER_CEMENT = 0.5877
R_CEMENT_ROCK = 0.3448

_W = ("water", 1480.0, 1000.0)
_S = ("steel", 5900.0, 7850.0)
_C = ("cement", 3000.0, 1900.0)
_R = ("rock", 4500.0, 2600.0)


def _medium(layers, thickness):
    return Medium(speed=tuple(l[1] for l in layers), thickness=tuple(thickness),
                  atten=tuple(0.0 for _ in layers), density=tuple(l[2] for l in layers),
                  names=tuple(l[0] for l in layers))


def card_c1() -> Card:
    """64x64 grid, 1 transmitter, 8 receivers, 256 samples at 10 MHz, 20 dB."""
    return Card(
        name="c1-plain-64x64",
        medium=_medium((_W, _S, _C), (10 * MM, 8 * MM)),
        grid=Grid(nx=64, nz=64, dx=0.5 * MM, dz=0.5 * MM, x0=-16 * MM),
        array=Array(tx_x=(0.0,), rx_offset=tuple((j - 3.5) * 5 * MM for j in range(8)), beta=8),
        acq=Acquisition(n_samples=256, fs=10 * MHZ, f_c=0.5 * MHZ, sigma_t=1.25 * US,
                        t_win=12 * US, oversample=64),
        prior=Prior(),
        phantom=PhantomSpec(seed=0, n_reflectors=5, amp_lo=0.5, amp_hi=1.0,
                            rows=(4, 46), cols=(8, 56), min_spacing=4,
                            interfaces=((20, R_WATER_STEEL), (36, R_STEEL_CEMENT))),
        snr_db=20.0, noise_seed=100, n_iter=20)


def card_c2() -> Card:
    """256x256 grid, 32 scan positions x 16 receivers, 2048 samples at 20 MHz, 15 dB."""
    return Card(
        name="c2-plain-256x256",
        medium=_medium((_W, _S, _C), (10 * MM, 8 * MM)),
        grid=Grid(nx=256, nz=256, dx=0.5 * MM, dz=0.5 * MM, x0=-64 * MM),
        array=Array(tx_x=tuple((-62 + 4 * i) * MM for i in range(32)),
                    rx_offset=tuple((j - 7.5) * 5 * MM for j in range(16)), beta=8),
        acq=Acquisition(n_samples=2048, fs=20 * MHZ, f_c=0.5 * MHZ, sigma_t=1.25 * US,
                        t_win=12 * US, oversample=32),
        prior=Prior(),
        phantom=PhantomSpec(seed=1, n_reflectors=40, amp_lo=0.3, amp_hi=1.0,
                            rows=(52, 250), cols=(16, 240), min_spacing=4,
                            interfaces=((20, R_WATER_STEEL), (36, R_STEEL_CEMENT)),
                            gap=(36, 2 * MM, 6 * MM, 0.2, 0.4,
                                 R_STEEL_WATER, R_WATER_CEMENT, R_STEEL_CEMENT)),
        snr_db=15.0, noise_seed=101, n_iter=50)


def card_c3() -> Card:
    """512x512 grid, four layers, 64 scan positions x 32 receivers, 4096 samples."""
    return Card(
        name="c3-precision-512x512",
        medium=_medium((_W, _S, _C, _R), (10 * MM, 8 * MM, 80 * MM)),
        grid=Grid(nx=512, nz=512, dx=0.5 * MM, dz=0.5 * MM, x0=-128 * MM),
        array=Array(tx_x=tuple((-126 + 4 * i) * MM for i in range(64)),
                    rx_offset=tuple((j - 15.5) * 5 * MM for j in range(32)), beta=8),
        acq=Acquisition(n_samples=4096, fs=20 * MHZ, f_c=0.5 * MHZ, sigma_t=1.25 * US,
                        t_win=12 * US, oversample=32),
        prior=Prior(),
        phantom=PhantomSpec(seed=2, n_reflectors=80, amp_lo=0.3, amp_hi=1.0,
                            rows=(52, 500), cols=(32, 480), min_spacing=4,
                            interfaces=((20, R_WATER_STEEL), (36, R_STEEL_CEMENT),
                                        (196, R_CEMENT_ROCK)),
                            gap=(36, 2 * MM, 6 * MM, 0.2, 0.4,
                                 R_STEEL_WATER, R_WATER_CEMENT, R_STEEL_CEMENT)),
        snr_db=15.0, noise_seed=102, n_iter=50)


def tiny_card(n_layers: int = 2, nx: int = 12, nz: int = 10, n_scans: int = 2,
              n_rx: int = 3, n_samples: int = 256, oversample: int = 8,
              beta: int = 8, seed: int = 7, atten: Optional[Tuple[float, ...]] = None) -> Card:
    """A small problem for tests whose oracle runs in well under a second.

    A 2 MHz pulse (t_0 = 3 us, 60 samples at 20 MHz) keeps the record short.
    Layers: water 1480 m/s / 2 mm, steel 5900 m/s / 3 mm, cement 3000 m/s.
    """
    layers = (_W, _S, _C, _R)[:n_layers]
    thick = (2 * MM, 3 * MM, 2 * MM)[:n_layers - 1]
    med = _medium(layers, thick)
    if atten is not None:
        med = Medium(speed=med.speed, thickness=med.thickness, atten=tuple(atten),
                     density=med.density, names=med.names)
    dx = 1 * MM
    x0 = -nx * dx / 2
    return Card(
        name=f"tiny-{n_layers}L-{nx}x{nz}",
        medium=med,
        grid=Grid(nx=nx, nz=nz, dx=dx, dz=0.5 * MM, x0=x0),
        array=Array(tx_x=tuple((-1.5 + 3 * i) * MM for i in range(n_scans)),
                    rx_offset=tuple((j - (n_rx - 1) / 2) * 2 * MM for j in range(n_rx)),
                    beta=beta),
        acq=Acquisition(n_samples=n_samples, fs=20 * MHZ, f_c=2 * MHZ, sigma_t=0.3 * US,
                        t_win=3 * US, oversample=oversample),
        prior=Prior(),
        phantom=PhantomSpec(seed=seed, n_reflectors=3, amp_lo=0.5, amp_hi=1.0,
                            rows=(2, nz - 1), cols=(1, nx - 1), min_spacing=2,
                            interfaces=()),
        snr_db=20.0, noise_seed=seed + 50, n_iter=10)


# attenuation of water and concrete, taken as the paper's per-Hz figures per
# MHz (Sec. 3), in s/m; steel and rock are left lossless
ALPHA_WATER = 2e-6
ALPHA_CEMENT = 30e-6


def attenuated_card(n_gamma: int = 16, nx: int = 12, nz: int = 16, oversample: int = 8,
                    n_scans: int = 2, n_rx: int = 3, seed: int = 7, storage: int = 0) -> Card:
    """tiny_card with three layers (water, steel, cement) and attenuation in
    water and cement; 16 rows reach 3 mm into the cement."""
    c = tiny_card(n_layers=3, nx=nx, nz=nz, n_scans=n_scans, n_rx=n_rx, oversample=oversample, seed=seed,
                  atten=(ALPHA_WATER, 0.0, ALPHA_CEMENT))
    acq = Acquisition(**{**asdict(c.acq), "n_gamma": n_gamma, "storage": storage})
    return Card(**{**{f: getattr(c, f) for f in c.__dataclass_fields__}, "acq": acq,
                   "name": f"attenuated-{nx}x{nz}-G{n_gamma}"})


def _reflectivity(z1: float, z2: float) -> float:
    # (Z2 - Z1)/(Z2 + Z1) of a phantom interface, Z = density * speed
    return (z2 - z1) / (z2 + z1)


def batch_cards(n: int = 48, seed: int = 11):
    """Seeded uneven problems for the batched workload: square grids of 128 to
    384 voxels a side (0.5 mm), three or four layers with seeded speeds and
    thicknesses (water / steel / cement / rock), 4 to 16 scan positions 4 mm
    apart, 8 to 32 receivers at 5 mm pitch, 1024 to 4096 samples at 20 MHz,
    point reflectors plus the interface rows, 15 dB, 20 to 50 iterations.
    Every transducer sits on the grid's half-voxel lattice."""
    import numpy as np
    rng = np.random.default_rng(seed)
    cards = []
    for i in range(n):
        side = int(rng.choice(np.arange(128, 385, 32)))
        n_layers = int(rng.integers(3, 5))
        c = (float(rng.uniform(1450, 1520)), float(rng.uniform(5800, 6000)),
             float(rng.uniform(2800, 3400)), float(rng.uniform(4200, 4800)))[:n_layers]
        rho = (1000.0, 7850.0, 1900.0, 2600.0)[:n_layers]
        depth = side * 0.5 * MM
        thick = [float(rng.uniform(8, 12)) * MM, float(rng.uniform(6, 10)) * MM]
        if n_layers == 4:
            thick.append(float(rng.uniform(0.3, 0.6)) * depth)
        names = ("water", "steel", "cement", "rock")[:n_layers]
        med = Medium(speed=c, thickness=tuple(thick), atten=(0.0,) * n_layers, density=rho, names=names)
        n_scans = int(rng.integers(4, 17))
        n_rx = int(rng.integers(8, 33))
        n_samples = int(rng.choice(np.arange(1024, 4097, 512)))
        tops = np.cumsum(thick)
        rows = [int(round(t / (0.5 * MM))) for t in tops]
        interfaces = tuple((r, round(_reflectivity(rho[k] * c[k], rho[k + 1] * c[k + 1]), 4))
                           for k, r in enumerate(rows) if r < side)
        cards.append(Card(
            name=f"b{i}-{side}x{side}-{n_layers}L-{n_scans}x{n_rx}-{n_samples}",
            medium=med,
            grid=Grid(nx=side, nz=side, dx=0.5 * MM, dz=0.5 * MM, x0=-side * 0.25 * MM),
            array=Array(tx_x=tuple((-2.0 * (n_scans - 1) + 4.0 * k) * MM for k in range(n_scans)),
                        rx_offset=tuple((j - (n_rx - 1) / 2) * 5 * MM for j in range(n_rx)), beta=8),
            acq=Acquisition(n_samples=n_samples, fs=20 * MHZ, f_c=0.5 * MHZ, sigma_t=1.25 * US,
                            t_win=12 * US, oversample=32),
            prior=Prior(),
            phantom=PhantomSpec(seed=1000 + i, n_reflectors=side // 8, amp_lo=0.3, amp_hi=1.0,
                                rows=(rows[1] + 4 if rows[1] + 4 < side - 4 else side // 2, side - 4),
                                cols=(8, side - 8), min_spacing=4, interfaces=interfaces),
            snr_db=15.0, noise_seed=2000 + i, n_iter=int(rng.integers(20, 51))))
    return cards


CARDS = {"c1": card_c1, "c2": card_c2, "c3": card_c3}
