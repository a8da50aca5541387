"""Pins of the oracle's time-of-day / date sun by astronomical and atmospheric facts that do not
come from its own formulas: solstice and equinox declinations, the extremes of the equation of
time, perihelion and aphelion distances, the geometry of solar noon, sunrise and symmetric hours,
the air mass at zenith, 60 degrees and the horizon, Rayleigh optical depths of the standard
atmosphere, and the reddening of a low sun."""
import math

import numpy as np
import pytest

from oracle import daylight as dl


def test_solstice_and_equinox_declinations():
    assert abs(math.degrees(dl.declination(172)) - 23.44) < 0.3     # June solstice
    assert abs(math.degrees(dl.declination(355)) + 23.44) < 0.3     # December solstice
    assert abs(math.degrees(dl.declination(80))) < 0.6              # March equinox
    assert abs(math.degrees(dl.declination(266))) < 0.8             # September equinox


def test_equation_of_time_extremes():
    eot = np.array([dl.equation_of_time_min(d) for d in range(1, 366)])
    assert abs(eot.max() - 16.4) < 0.7 and 295 <= np.argmax(eot) + 1 <= 315      # early November
    assert abs(eot.min() + 14.2) < 0.7 and 35 <= np.argmin(eot) + 1 <= 50        # mid February


def test_earth_sun_distance_extremes():
    # perihelion (early January) at 0.98329 AU, aphelion (early July) at 1.01671 AU
    assert abs(dl.distance_factor(3) - 1 / 0.98329**2) < 2e-3
    assert abs(dl.distance_factor(185) - 1 / 1.01671**2) < 2e-3


def _tst_params(day, tst_hours, lat, psi=90.0):
    """Parameters whose clock time gives true solar time tst_hours at longitude 0, UTC."""
    return dl.Daylight(day_of_year=day, clock_hours=tst_hours - dl.equation_of_time_min(day) / 60.0,
                       utc_offset_hours=0.0, latitude_deg=lat, longitude_deg=0.0, scene_x_azimuth_deg=psi)


@pytest.mark.parametrize("lat,day", [(49.14, 172), (49.14, 355), (-33.9, 20), (10.0, 80)])
def test_solar_noon_and_symmetric_hours(lat, day):
    el, az, h = dl.solar_position(_tst_params(day, 12.0, lat))
    dec = math.degrees(dl.declination(day))
    assert abs(h) < 1e-9
    assert abs(el - (90.0 - abs(lat - dec))) < 1e-9
    assert abs(az - (180.0 if lat > dec else 0.0)) % 360.0 < 1e-6
    for dh in (1.5, 4.0):
        e1, a1, _ = dl.solar_position(_tst_params(day, 12.0 - dh, lat))
        e2, a2, _ = dl.solar_position(_tst_params(day, 12.0 + dh, lat))
        assert abs(e1 - e2) < 1e-9 and abs((a1 + a2) % 360.0) < 1e-6


def test_equinox_sunrise_in_the_east():
    p = _tst_params(80, 6.0, 49.14)
    p.day_of_year = 80
    el, az, _ = dl.solar_position(p)
    dec = math.degrees(dl.declination(80))
    assert abs(el) < abs(dec) + 0.3 and abs(az - 90.0) < 1.0


def test_scene_frame_of_the_direction():
    """+x pointing east (azimuth 90): noon sun lies in the y-z plane toward -y (south); a
    morning sun has +x (east). With +x pointing north the noon sun is toward -x."""
    d, _, _ = dl.sun(_tst_params(172, 12.0, 49.14, psi=90.0), 4)
    assert abs(d[0]) < 1e-12 and d[1] < 0 and d[2] > 0 and abs(np.linalg.norm(d) - 1) < 1e-12
    d, _, _ = dl.sun(_tst_params(172, 9.0, 49.14, psi=90.0), 4)
    assert d[0] > 0.3
    d, _, _ = dl.sun(_tst_params(172, 12.0, 49.14, psi=0.0), 4)
    assert d[0] < 0 and abs(d[1]) < 1e-12


def test_air_mass_values():
    assert abs(dl.air_mass(0.0) - 1.0) < 1e-3
    assert abs(dl.air_mass(60.0) - 2.0) < 0.01          # close to sec(60) away from the horizon
    assert abs(dl.air_mass(90.0) - 38.0) < 0.2          # the horizon value of the Kasten-Young fit


def test_rayleigh_optical_depth_of_the_standard_atmosphere():
    assert abs(dl.rayleigh_tau(550.0) - 0.0973) < 0.002
    assert abs(dl.rayleigh_tau(400.0) - 0.36) < 0.01
    r = dl.rayleigh_tau(400.0) / dl.rayleigh_tau(800.0)
    assert 16.0 < r < 17.5                                 # close to the lambda^-4 law
    assert abs(dl.rayleigh_tau(550.0, 0.5) - 0.5 * dl.rayleigh_tau(550.0)) < 1e-15


def test_spectrum_zenith_sun_and_reddening():
    # zenith sun at mean distance: blackbody times one air mass of Rayleigh transmittance
    p = dl.Daylight(day_of_year=172, latitude_deg=23.44, longitude_deg=0.0, utc_offset_hours=0.0)
    p.clock_hours = 12.0 - dl.equation_of_time_min(172) / 60.0
    p.latitude_deg = math.degrees(dl.declination(172))
    d, E, info = dl.sun(p, 40)
    assert info["elevation_deg"] > 89.999 and abs(info["air_mass"] - 1.0) < 1e-3
    lam = 380 + (np.arange(40) + 0.5) * 10
    assert np.all(E > 0)
    # E at 555-ish normalised close to the transmittance there
    j = np.argmin(np.abs(lam - 555))
    assert abs(E[j] / info["distance_factor"] - math.exp(-0.0973)) < 0.02
    # a lower sun is redder: E(700)/E(450) grows as the sun sinks, and E vanishes below the horizon
    pts = []
    for hh in (12.0, 15.0, 17.0, 18.5, 19.5, 20.5, 21.3):
        p2 = dl.Daylight(day_of_year=172, clock_hours=hh, utc_offset_hours=2.0)
        _, E2, inf2 = dl.sun(p2, 40)
        if inf2["elevation_deg"] > 0:
            pts.append((inf2["elevation_deg"], E2[np.argmin(np.abs(lam - 700))] / E2[np.argmin(np.abs(lam - 450))]))
    pts.sort(reverse=True)
    ratios = [r for _, r in pts]
    assert len(ratios) >= 5 and np.all(np.diff(ratios) > 0) and pts[-1][0] < 5.0
    _, E3, inf3 = dl.sun(dl.Daylight(day_of_year=172, clock_hours=1.0, utc_offset_hours=2.0), 8)
    assert inf3["elevation_deg"] < 0 and np.all(E3 == 0)
