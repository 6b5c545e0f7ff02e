"""Seeded synthetic workloads (inputs only; no part of the method).

The paper's preconditioner benchmark uses Planck inverse-noise maps and masks
at N_side = 2048 that are not available here.  These generators stand in for
their structure: smooth scan-strategy hit counts, per-pixel noise and masked
regions, at the resolutions the paper benchmarks (lmax from 64 to 3000, tile
size k = 8).  Every map is a function of the pixel colatitude/longitude arrays
passed in, so any grid implementation can feed the same values to both sides.

Beam: Gaussian with FWHM = f * Delta, Delta = sqrt(4 pi / Npix) (the mean
pixel spacing), b_l = exp(-l (l+1) sigma^2 / 2), sigma = FWHM / sqrt(8 ln 2),
truncated at radius R = 3 FWHM.  Prior: d_l = (l+1)^2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Config:
    name: str
    lmax: int
    k: int
    fwhm_pix: float
    ninv_kind: str
    seed: int


CONFIGS = {
    "lmax64": Config("lmax64", 64, 8, 3.0, "uniform", 101),
    "lmax512": Config("lmax512", 512, 8, 3.0, "dipole_mask", 202),
    "lmax1500": Config("lmax1500", 1500, 8, 3.0, "dipole_mask", 303),
    "lmax3000": Config("lmax3000", 3000, 8, 3.0, "scan_lognormal", 404),
}

BATCH_LMAX = (256, 512, 1024, 2048)


def pixel_spacing(npix: int) -> float:
    return math.sqrt(4.0 * math.pi / npix)


def gaussian_beam(lmax: int, npix: int, fwhm_pix: float):
    """(b_l, R): Gaussian beam of FWHM = fwhm_pix mean pixel spacings and its
    truncation radius R = 3 FWHM (radians)."""
    fwhm = fwhm_pix * pixel_spacing(npix)
    sigma = fwhm / math.sqrt(8.0 * math.log(2.0))
    ell = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * ell * (ell + 1.0) * sigma * sigma), 3.0 * fwhm


def prior(lmax: int):
    """d_l = (l+1)^2."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    return (ell + 1.0) ** 2


def _unit(theta, phi):
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=-1)


def ninv_uniform(theta, phi, seed: int):
    """i.i.d. U[0.5, 2] per pixel."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.5, 2.0, size=np.shape(theta))


def ninv_dipole_mask(theta, phi, seed: int):
    """10^u with u = clip(0.8 n.d + 0.2 eps, -1, 1), d at (60 deg, 45 deg):
    values in [0.1, 10]; zero in the band |theta - 90 deg| < 10 deg."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = rng.standard_normal(np.shape(theta))
    d = _unit(np.deg2rad(60.0), np.deg2rad(45.0))
    u = np.clip(0.8 * (_unit(theta, phi) @ d) + 0.2 * eps, -1.0, 1.0)
    out = 10.0 ** u
    out[np.abs(theta - 0.5 * np.pi) < np.deg2rad(10.0)] = 0.0
    return out


def ninv_scan_lognormal(theta, phi, seed: int):
    """exp(0.5 eps) * s(n) * mask.  s = (1 + 0.5 cos 32 lam)(0.5 + |cos beta|) in a
    frame whose pole is at (60 deg, 0), lam/beta its longitude/latitude; the mask
    removes |n.g| < 0.2 with g at (60 deg, 120 deg), i.e. 20% of the sky."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = rng.standard_normal(np.shape(theta))
    n = _unit(theta, phi)
    pole = _unit(np.deg2rad(60.0), 0.0)
    # orthonormal frame (e1, e2, pole)
    e1 = np.cross(np.array([0.0, 0.0, 1.0]), pole)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(pole, e1)
    zc = np.clip(n @ pole, -1.0, 1.0)
    lam = np.arctan2(n @ e2, n @ e1)
    cos_beta = np.sqrt(np.maximum(0.0, 1.0 - zc * zc))
    s = (1.0 + 0.5 * np.cos(32.0 * lam)) * (0.5 + cos_beta)
    g = _unit(np.deg2rad(60.0), np.deg2rad(120.0))
    mask = np.abs(n @ g) >= 0.2
    return np.exp(0.5 * eps) * s * mask


def ninv_for(cfg: Config, theta, phi):
    fn = {"uniform": ninv_uniform, "dipole_mask": ninv_dipole_mask,
          "scan_lognormal": ninv_scan_lognormal}[cfg.ninv_kind]
    return fn(theta, phi, cfg.seed)


def batch_problem(p: int):
    """Problem p of the 32-problem batch: lmax, FWHM in pixels, mask fraction,
    mask centre and seed.  N^-1 = U[0.5, 2] times a mask |n.g_p| < f_p."""
    rng = np.random.Generator(np.random.PCG64(5000 + p))
    fwhm = rng.uniform(2.0, 5.0)
    frac = rng.uniform(0.0, 0.3)
    v = rng.standard_normal(3)
    v /= np.linalg.norm(v)
    return {"lmax": BATCH_LMAX[p % 4], "fwhm_pix": fwhm, "mask_frac": frac,
            "g": v, "seed": 5000 + p}


def ninv_batch(theta, phi, prob):
    rng = np.random.Generator(np.random.PCG64(prob["seed"] + 100000))
    base = rng.uniform(0.5, 2.0, size=np.shape(theta))
    n = _unit(theta, phi)
    return base * (np.abs(n @ prob["g"]) >= prob["mask_frac"])
