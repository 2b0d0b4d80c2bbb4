"""Seeded synthetic workloads: grids, initial fields, currents and susceptibilities.

This module holds no arithmetic of the method -- only the workload recipes (the paper's laser and plasma
set-ups in normalised units) and seeded random draws.  Both the oracle-side tests and the GPU side take
their inputs from here.

Units: normalised with omega_r = omega_0 (section 1 conventions): lengths in c/omega_0 = lambda_0/(2 pi),
times in 1/omega_0, k0 = 1, chi = n/n_c.  lambda_0 = 0.8 um throughout, so 1 um = 2 pi / 0.8 units.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

UM = 2 * math.pi / 0.8          # one micrometre in units of c/omega_0 (lambda_0 = 0.8 um)
LAMBDA0 = 2 * math.pi           # the laser wavelength in the same units


@dataclass
class Workload:
    """A list of independent problems (one grid + one mode each) and the step count."""
    name: str
    kind: int                    # 0 Maxwell, 1 envelope
    nz: List[int]
    nr: List[int]
    m: List[int]
    fd_order: List[int]
    taylor_order: int
    dz: float
    dr: float
    dt: float
    steps: int
    k0: float = 1.0
    seed: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.m)

    def cells(self) -> int:
        return int(sum(a * b for a, b in zip(self.nz, self.nr)))

    def problems(self):
        from .binding import Problem
        return [Problem(nz=self.nz[p], nr=self.nr[p], m=self.m[p], fd_order=self.fd_order[p],
                        taylor_order=self.taylor_order, dz=self.dz, dr=self.dr, dt=self.dt, k0=self.k0,
                        kind=self.kind) for p in range(self.n)]

    def shrink(self, nz: Optional[int] = None, nr: Optional[int] = None, steps: Optional[int] = None) -> "Workload":
        return replace(self, nz=[nz or a for a in self.nz], nr=[nr or b for b in self.nr],
                       steps=steps if steps is not None else self.steps)


# ---------------------------------------------------------------------------------------------------
# The five workloads (vacuum pulse; current-driven solve; envelope in plasma; uneven batch; LWFA scale)
# ---------------------------------------------------------------------------------------------------
def vacuum_pulse() -> Workload:
    """m = 1 Gaussian pulse in vacuum, 256 x 64, order 8, 100 steps at dt = dz (Taylor order 12)."""
    dz = LAMBDA0 / 20
    return Workload("vacuum_pulse_m1_256x64_o8", 0, [256], [64], [1], [8], 12, dz, 2 * dz, dz, 100, seed=1,
                    extra=dict(w0=8 * LAMBDA0, ctau=1.5 * UM, zc=3.0 * UM, a0=1.0, noise=1e-6))


def current_driven() -> Workload:
    """Modes m = 0, 1 on 2048 x 256, order 16, 500 steps at dt = dz/2 (Taylor order 8), driven by a
    Gaussian electron bunch moving at c on the axis plus white-noise current."""
    dz = LAMBDA0 / 20
    return Workload("current_driven_m01_2048x256_o16", 0, [2048, 2048], [256, 256], [0, 1], [16, 16], 8, dz, 2 * dz,
                    0.5 * dz, 500, seed=2, extra=dict(sigz=2.0 * UM, sigr=1.0 * UM, nb=0.01, noise=1e-3))


def envelope_plasma() -> Workload:
    """Envelope a (a0 = 2, w0 = 20 um, 30 fs) on 4096 x 512 in chi = 1e-3 (1 + 5% smooth modulation),
    order 8, 2000 steps at dt = dz/2 (Taylor order 4), dz = lambda/5, dr = 0.2 um."""
    dz = LAMBDA0 / 5
    return Workload("envelope_plasma_4096x512_o8", 1, [4096], [512], [0], [8], 4, dz, 0.2 * UM, 0.5 * dz, 2000,
                    seed=3, extra=dict(a0=2.0, w0=20 * UM, ctau=9.0 * UM, zc=100 * UM, chi0=1e-3, mod=0.05))


def batched_uneven(n: int = 64) -> Workload:
    """n independent problems with uneven grids (nz in [512, 4096], nr in [64, 512]), modes 0..2 and
    orders 8..32, 200 steps at dt = dz/2 (Taylor order 8)."""
    nz, nr, m, order = [], [], [], []
    for p in range(n):
        r = np.random.default_rng(4000 + p)
        nz.append(int(r.integers(512, 4097)))
        nr.append(int(r.integers(64, 513)))
        m.append(int(r.integers(0, 3)))
        order.append(int(2 * r.integers(4, 17)))
    dz = LAMBDA0 / 20
    return Workload("batched_uneven_64", 0, nz, nr, m, order, 8, dz, 2 * dz, 0.5 * dz, 200, seed=4,
                    extra=dict(sigz=2.0 * UM, sigr=1.0 * UM, nb=0.01, noise=1e-3, w0=8 * LAMBDA0, a0=1.0,
                                                                       ctau=1.5 * UM))


def lwfa_scale() -> Workload:
    """Modes m = 0, 1, 2 on 8192 x 1024, order 32, 1000 steps at dt = dz/2 (Taylor order 8);
    dz = 0.032 um, dr = 0.16 um; Gaussian pulse a0 = 4, w0 = 15 um, tau = 10 um / c."""
    dz, dr = 0.032 * UM, 0.16 * UM
    return Workload("lwfa_m012_8192x1024_o32", 0, [8192] * 3, [1024] * 3, [0, 1, 2], [32] * 3, 8, dz, dr, 0.5 * dz,
                    1000, seed=5, extra=dict(w0=15 * UM, ctau=10 * UM, zc=60 * UM, a0=4.0, sigz=2.0 * UM,
                                             sigr=1.0 * UM, nb=0.01, noise=1e-3))


WORKLOADS = {"vacuum_pulse": vacuum_pulse, "current_driven": current_driven, "envelope_plasma": envelope_plasma,
             "batched_uneven": batched_uneven, "lwfa_scale": lwfa_scale}


# ---------------------------------------------------------------------------------------------------
# Field and source recipes (numpy, complex128 / float64)
# ---------------------------------------------------------------------------------------------------
def _positions(nz, nr, dz, dr):
    """Sampling points of the six components: rho-staggered rows sit at k*dr, primary rows at (k+1/2)dr;
    z-staggered columns at (i-1/2)dz, primary at i*dz (E_rho, E_theta, E_z, B_rho, B_theta, B_z)."""
    rp, rs = (np.arange(nr) + 0.5) * dr, np.arange(nr) * dr
    zp, zs = np.arange(nz) * dz, (np.arange(nz) - 0.5) * dz
    return [(rs, zp), (rp, zp), (rp, zs), (rp, zs), (rs, zs), (rs, zp)]


def gaussian_pulse(nz, nr, m, dz, dr, w0, ctau, zc, a0, k0=1.0) -> np.ndarray:
    """x-polarised pulse E_x = B_y = a0 exp(-rho^2/w0^2) exp(-((z-zc)/ctau)^2) cos(k0 (z-zc)) at focus,
    with the first-order longitudinal components that make it divergence free, projected on azimuthal
    mode m (only m = 1 is non-zero: E_rho = E_x, E_theta = i E_x, B_rho = -i B_y, B_theta = B_y)."""
    psi = np.zeros((6, nr, nz), np.complex128)
    if m != 1:
        return psi
    for c, (r, z) in enumerate(_positions(nz, nr, dz, dr)):
        R, Z = np.meshgrid(r, z, indexing="ij")
        env = a0 * np.exp(-(R / w0) ** 2 - ((Z - zc) / ctau) ** 2)
        cos, sin = np.cos(k0 * (Z - zc)), np.sin(k0 * (Z - zc))
        lon = 2 * R / (k0 * w0 ** 2) * env * sin
        psi[c] = {0: env * cos, 1: 1j * env * cos, 2: lon, 3: -1j * env * cos, 4: env * cos, 5: -1j * lon}[c]
    return psi


def noise(shape, amplitude, rng, real_only=False) -> np.ndarray:
    x = rng.uniform(-1.0, 1.0, shape)
    if real_only:
        return amplitude * x.astype(np.complex128)
    return amplitude * (x + 1j * rng.uniform(-1.0, 1.0, shape))


def initial_fields(w: Workload, p: int, rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """Initial Maxwell state of problem p: the Gaussian pulse (when the workload defines one) plus the
    seeded uniform noise of the workload (m = 0: real part only)."""
    e = w.extra
    nz, nr, m = w.nz[p], w.nr[p], w.m[p]
    if "w0" in e:
        w0 = min(e["w0"], nr * w.dr / 3)
        psi = gaussian_pulse(nz, nr, m, w.dz, w.dr, w0, e["ctau"], e.get("zc", 0.3 * nz * w.dz), e["a0"])
    else:
        psi = np.zeros((6, nr, nz), np.complex128)
    amp = e.get("noise", 0.0) if "w0" in e and "nb" not in e else 0.0
    if amp:
        rng = rng or np.random.default_rng(w.seed * 1000 + p)
        psi += noise(psi.shape, amp, rng, real_only=(m == 0))
    return psi


def bunch_current(w: Workload, p: int, step: int, rng: np.random.Generator) -> np.ndarray:
    """Current at t = (step + 1/2) dt: a Gaussian charge bunch (sigma_z, sigma_r, density n_b) moving at c
    along the axis (J_z, mode 0 only), plus uniform white noise of relative amplitude `noise` on all three
    components (mode 0: real part only).  J_rho, J_theta on (rho_k, z_i); J_z on (rho_k, z_i - dz/2)."""
    e = w.extra
    nz, nr, m = w.nz[p], w.nr[p], w.m[p]
    j = np.zeros((3, nr, nz), np.complex128)
    t = (step + 0.5) * w.dt
    rp = (np.arange(nr) + 0.5) * w.dr
    zs = (np.arange(nz) - 0.5) * w.dz
    zb = 0.25 * nz * w.dz + t
    if m == 0:
        j[2] = -e["nb"] * np.exp(-((zs[None, :] - zb) ** 2) / (2 * e["sigz"] ** 2) - rp[:, None] ** 2 / (2 * e["sigr"] ** 2))
    j += noise(j.shape, e["noise"] * e["nb"], rng, real_only=(m == 0))
    return j


def currents(w: Workload, p: int, steps: int, first_step: int = 0) -> np.ndarray:
    """[steps, 3, nr, nz] currents of problem p for steps first_step .. first_step + steps - 1."""
    rng = np.random.default_rng([w.seed, p, first_step])
    return np.stack([bunch_current(w, p, first_step + s, rng) for s in range(steps)])


def envelope_initial(w: Workload, p: int = 0):
    """a = a0 exp(-rho^2/w0^2) exp(-((z-zc)/ctau)^2), a~ = -d a/dz (forward-moving envelope)."""
    e = w.extra
    nz, nr = w.nz[p], w.nr[p]
    rp = (np.arange(nr) + 0.5) * w.dr
    z = np.arange(nz) * w.dz
    zc = min(e["zc"], 0.5 * nz * w.dz)
    ctau = min(e["ctau"], 0.1 * nz * w.dz)
    w0 = min(e["w0"], nr * w.dr / 3)
    g = np.exp(-(rp[:, None] / w0) ** 2 - ((z[None, :] - zc) / ctau) ** 2)
    a = (e["a0"] * g).astype(np.complex128)
    at = (2 * (z[None, :] - zc) / ctau ** 2 * a).astype(np.complex128)
    return a, at


def envelope_chi(w: Workload, p: int = 0) -> np.ndarray:
    """chi = chi0 (1 + mod g), g a seeded sum of 8 random low-wavenumber cosines (lambda_z >= 20 um,
    lambda_r >= 10 um) normalised to max|g| = 1."""
    e = w.extra
    nz, nr = w.nz[p], w.nr[p]
    rng = np.random.default_rng(w.seed * 7919 + p)
    rp = (np.arange(nr) + 0.5) * w.dr
    z = np.arange(nz) * w.dz
    g = np.zeros((nr, nz))
    for _ in range(8):
        kz = rng.uniform(0, 2 * math.pi / (20 * UM))
        kr = rng.uniform(0, 2 * math.pi / (10 * UM))
        ph = rng.uniform(0, 2 * math.pi, 2)
        g += np.cos(kr * rp[:, None] + ph[0]) * np.cos(kz * z[None, :] + ph[1])
    g /= np.max(np.abs(g))
    return e["chi0"] * (1 + e["mod"] * g)


# ---------------------------------------------------------------------------------------------------
# Counter-based current of the captured time loop (fdetd_step_graph, FDETD_JGEN_BUNCH): the bunch recipe
# above with its noise drawn by SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
# generators", OOPSLA 2014) from a counter, so that the library's generator kernel and this host copy
# produce the same values without sharing code.
# ---------------------------------------------------------------------------------------------------
SPLITMIX_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(z):
    """The SplitMix64 output function (the generator's mixing of its state), on uint64 values (arithmetic
    modulo 2^64)."""
    with np.errstate(over="ignore"):
        z = np.asarray(z, dtype=np.uint64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def counter_key(seed: int, step: int, problem: int):
    """Stream key of one (seed, step, problem): h0 = mix(seed + g), h1 = mix(h0 + (step + 1) g),
    h2 = mix(h1 + (problem + 1) g), g the SplitMix64 increment."""
    with np.errstate(over="ignore"):
        h = splitmix64(np.uint64(seed % 2 ** 64) + SPLITMIX_GAMMA)
        h = splitmix64(h + np.uint64(step + 1) * SPLITMIX_GAMMA)
        return splitmix64(h + np.uint64(problem + 1) * SPLITMIX_GAMMA)


def counter_uniform(seed: int, step: int, problem: int, shape) -> np.ndarray:
    """U[-1, 1) values number v = 0 .. prod(shape) - 1 of a stream: mix(key + (v + 1) g), top 53 bits."""
    key = counter_key(seed, step, problem)
    n = int(np.prod(shape))
    v = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        u = splitmix64(key + v * SPLITMIX_GAMMA)
    return ((u >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0).reshape(shape)


def graph_bunch_current(w: Workload, p: int, step: int, seed: int) -> np.ndarray:
    """Current of step `step` (t = (step + 1/2) dt) as the library's FDETD_JGEN_BUNCH generator forms it:
    uniform noise of amplitude noise * n_b on the real and imaginary parts of J_rho, J_theta, J_z (value
    number ((c nr + k) nz + i) 2 + part of the stream (seed, step, p); mode 0 keeps the real parts only),
    plus on J_z of mode 0 the Gaussian bunch -n_b exp(-(z - z_b)^2 / (2 sigma_z^2) - rho^2 / (2 sigma_r^2)),
    z_b = 0.25 nz dz + t, at (rho_k, z_i - dz/2)."""
    e = w.extra
    nz, nr, m = w.nz[p], w.nr[p], w.m[p]
    u = counter_uniform(seed, step, p, (3, nr, nz, 2)) * (e["noise"] * e["nb"])
    j = u[..., 0] + 1j * (u[..., 1] if m != 0 else 0.0)
    if m == 0:
        t = (step + 0.5) * w.dt
        rp = (np.arange(nr) + 0.5) * w.dr
        zs = (np.arange(nz) - 0.5) * w.dz
        zb = 0.25 * nz * w.dz + t
        j[2] += -e["nb"] * np.exp(-((zs[None, :] - zb) ** 2) / (2 * e["sigz"] ** 2) - rp[:, None] ** 2 / (2 * e["sigr"] ** 2))
    return j
