"""The library's daylight sun (host computation behind the C ABI, no GPU needed) against the
oracle's FP64 daylight model: direction within 2e-6, geometry within 1e-4 degrees, and the
irradiance within 2e-6 relative (FP32 rounding of FP64 values), over dates, times, sites, scene
orientations, temperatures and pressures; out-of-range parameters are refused."""
import math

import numpy as np
import pytest

from oracle import daylight as dl

CASES = [
    dict(day_of_year=172, clock_hours=14.5, utc_offset_hours=2.0, latitude_deg=49.14, longitude_deg=2.38,
         scene_x_azimuth_deg=90.0),
    dict(day_of_year=355, clock_hours=10.25, utc_offset_hours=1.0, latitude_deg=49.14, longitude_deg=2.38,
         scene_x_azimuth_deg=90.0),
    dict(day_of_year=80, clock_hours=7.0, utc_offset_hours=0.0, latitude_deg=0.0, longitude_deg=-10.0,
         scene_x_azimuth_deg=30.0, temperature_k=6500.0),
    dict(day_of_year=20, clock_hours=18.7, utc_offset_hours=10.0, latitude_deg=-33.9, longitude_deg=151.2,
         scene_x_azimuth_deg=-135.0, pressure_ratio=0.7),
    dict(day_of_year=300, clock_hours=16.9, utc_offset_hours=-5.0, latitude_deg=64.1, longitude_deg=-21.9,
         scene_x_azimuth_deg=0.0),
    dict(day_of_year=366, clock_hours=23.0, utc_offset_hours=0.0, latitude_deg=70.0, longitude_deg=0.0,
         scene_x_azimuth_deg=45.0),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("B", [8, 40, 80])
def test_library_daylight_matches_oracle(case, B):
    import paper_1912_04000_amd as sd
    kw = CASES[case]
    d, E, info = sd.daylight_sun(sd.daylight(**kw), B, 380.0, 780.0)
    # the oracle takes the parameters as the library receives them (FP32)
    kw32 = {k: (v if isinstance(v, int) else float(np.float32(v))) for k, v in kw.items()}
    od, oE, oinfo = dl.sun(dl.Daylight(**kw32), B, 380.0, 780.0)
    np.testing.assert_allclose(d, od, atol=2e-6)
    assert abs(info["elevation_deg"] - oinfo["elevation_deg"]) < 1e-4
    assert abs((info["azimuth_deg"] - oinfo["azimuth_deg"] + 180.0) % 360.0 - 180.0) < 1e-4
    assert abs(info["distance_factor"] - oinfo["distance_factor"]) < 1e-6
    if oinfo["elevation_deg"] > 0:
        assert abs(info["air_mass"] - oinfo["air_mass"]) <= 2e-6 * oinfo["air_mass"]
        np.testing.assert_allclose(E, oE, rtol=2e-6)
    else:
        assert math.isinf(info["air_mass"]) and np.all(E == 0)


@pytest.mark.parametrize("field,value", [("day_of_year", 0), ("day_of_year", 367), ("clock_hours", 25.0),
                                         ("latitude_deg", 91.0), ("longitude_deg", 181.0),
                                         ("temperature_k", 10.0), ("pressure_ratio", -1.0),
                                         ("scene_x_azimuth_deg", float("nan"))])
def test_out_of_range_parameters_are_refused(field, value):
    import paper_1912_04000_amd as sd
    p = sd.daylight(**{field: value})
    with pytest.raises(sd.SddError) as e:
        sd.daylight_sun(p, 8)
    assert e.value.code == -1
