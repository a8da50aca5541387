"""Time-of-day and date dependent sun, FP64 -- TEST INFRASTRUCTURE ONLY (oracle).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this module; the renderer never does. It is the plain statement of what the library's daylight
model computes.

Section 3 of the paper: the sun is a plane wave; its spectrum as seen from the ground changes
with the hour (the incidence angle through the atmosphere: sunsets are redder) and with the date
(the Earth-Sun distance along the elliptic orbit), and a plausible spectrum follows from
Rayleigh scattering theory. The paper gives no constants; this reading uses published ones:
  * solar declination, equation of time and inverse squared Earth-Sun distance: the Fourier
    series of J. W. Spencer (Search 2(5), 1971) in the day angle G = 2 pi (d - 1) / 365;
  * the sun's position from the site latitude and the hour angle of true solar time;
  * relative optical air mass: Kasten and Young (Applied Optics 28(22), 1989);
  * Rayleigh optical depth of the standard atmosphere at sea level: Hansen and Travis (Space
    Sci. Rev. 16, 1974), tau(l) = 0.008569 l^-4 (1 + 0.0113 l^-2 + 0.00013 l^-4), l in um,
    scaled by the surface pressure ratio;
  * extraterrestrial spectrum: a blackbody of temperature T normalised to 1 at 555 nm.
Spectrum at bin centre l_j (nm): E_j = B(l_j, T) / B(555, T) * (r0/r)^2 * exp(-tau(l_j) m p)
when the sun is above the horizon, else 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

H_PLANCK = 6.62607015e-34
C_LIGHT = 299792458.0
K_BOLTZMANN = 1.380649e-23


@dataclass
class Daylight:
    day_of_year: int = 172
    clock_hours: float = 12.0
    utc_offset_hours: float = 0.0
    latitude_deg: float = 49.14
    longitude_deg: float = 2.38
    scene_x_azimuth_deg: float = 90.0   # compass azimuth (clockwise from north) of the scene's +x axis
    temperature_k: float = 5778.0
    pressure_ratio: float = 1.0


def day_angle(d):
    return 2.0 * math.pi * (d - 1) / 365.0


def declination(d):
    """Solar declination (radians), Spencer 1971."""
    g = day_angle(d)
    return (0.006918 - 0.399912 * math.cos(g) + 0.070257 * math.sin(g) - 0.006758 * math.cos(2 * g)
            + 0.000907 * math.sin(2 * g) - 0.002697 * math.cos(3 * g) + 0.00148 * math.sin(3 * g))


def equation_of_time_min(d):
    """Equation of time (minutes), Spencer 1971."""
    g = day_angle(d)
    return 229.18 * (0.000075 + 0.001868 * math.cos(g) - 0.032077 * math.sin(g) - 0.014615 * math.cos(2 * g)
                     - 0.040849 * math.sin(2 * g))


def distance_factor(d):
    """(r0 / r)^2, Spencer 1971."""
    g = day_angle(d)
    return (1.000110 + 0.034221 * math.cos(g) + 0.001280 * math.sin(g) + 0.000719 * math.cos(2 * g)
            + 0.000077 * math.sin(2 * g))


def air_mass(zenith_deg):
    """Relative optical air mass, Kasten and Young 1989 (zenith angle in degrees, up to 90)."""
    z = float(zenith_deg)
    return 1.0 / (math.cos(math.radians(z)) + 0.50572 * (96.07995 - z) ** -1.6364)


def rayleigh_tau(lambda_nm, pressure_ratio=1.0):
    """Rayleigh optical depth, Hansen and Travis 1974."""
    l = np.asarray(lambda_nm, dtype=np.float64) * 1e-3
    return pressure_ratio * 0.008569 * l**-4 * (1.0 + 0.0113 * l**-2 + 0.00013 * l**-4)


def planck(lambda_nm, t):
    lam = np.asarray(lambda_nm, dtype=np.float64) * 1e-9
    return 2.0 * H_PLANCK * C_LIGHT**2 / lam**5 / np.expm1(H_PLANCK * C_LIGHT / (lam * K_BOLTZMANN * t))


def solar_position(p: Daylight):
    """(elevation, compass azimuth) in degrees and the hour angle (degrees) at the site."""
    tst = p.clock_hours * 60.0 + equation_of_time_min(p.day_of_year) + 4.0 * p.longitude_deg - 60.0 * p.utc_offset_hours
    h = math.radians(tst / 4.0 - 180.0)
    phi, dec = math.radians(p.latitude_deg), declination(p.day_of_year)
    sin_el = math.sin(phi) * math.sin(dec) + math.cos(phi) * math.cos(dec) * math.cos(h)
    el = math.asin(max(-1.0, min(1.0, sin_el)))
    # azimuth measured from south toward west, then from north clockwise
    az_s = math.atan2(math.sin(h), math.cos(h) * math.sin(phi) - math.tan(dec) * math.cos(phi))
    az = (math.degrees(az_s) + 180.0) % 360.0
    return math.degrees(el), az, math.degrees(h)


def sun(p: Daylight, n_bins: int, lambda_min_nm: float = 380.0, lambda_max_nm: float = 780.0):
    """Direction toward the sun in the scene frame (+z up, +x at compass azimuth
    scene_x_azimuth_deg, +y = z x x) and the spectrum E [n_bins]; plus a dict of the geometry."""
    el, az, _ = solar_position(p)
    e, a = math.radians(el), math.radians(az)
    east, north, up = math.cos(e) * math.sin(a), math.cos(e) * math.cos(a), math.sin(e)
    psi = math.radians(p.scene_x_azimuth_deg)
    d = np.array([east * math.sin(psi) + north * math.cos(psi), -east * math.cos(psi) + north * math.sin(psi), up])
    j = np.arange(n_bins, dtype=np.float64)
    lam = lambda_min_nm + (j + 0.5) * (lambda_max_nm - lambda_min_nm) / n_bins
    zen = 90.0 - el
    info = dict(elevation_deg=el, azimuth_deg=az, distance_factor=distance_factor(p.day_of_year))
    if el <= 0.0:
        info["air_mass"] = math.inf
        return d, np.zeros(n_bins), info
    m = air_mass(zen)
    info["air_mass"] = m
    E = planck(lam, p.temperature_k) / planck(555.0, p.temperature_k) * info["distance_factor"] * np.exp(
        -rayleigh_tau(lam, p.pressure_ratio) * m)
    return d, E, info
