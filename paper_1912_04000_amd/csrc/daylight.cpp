// Time-of-day and date dependent sun of libspecdd (host setup, like the scene build).
//
// Section 3 of the paper: the sun is a plane wave whose spectrum at the ground depends on the
// hour (the path through the atmosphere; sunsets are redder) and on the date (the Earth-Sun
// distance along the elliptic orbit), and Rayleigh scattering theory gives a plausible spectrum.
// Constants (the paper gives none):
//   - declination, equation of time, (r0/r)^2: Fourier series in the day angle
//     G = 2 pi (d - 1) / 365 (J. W. Spencer, 1971);
//   - position from the latitude and the hour angle of true solar time
//     (clock time + equation of time + 4 min per degree of longitude - the zone offset);
//   - air mass m(z) = 1 / (cos z + 0.50572 (96.07995 - z)^-1.6364), z in degrees (Kasten, Young
//     1989);
//   - Rayleigh optical depth tau(l) = 0.008569 l^-4 (1 + 0.0113 l^-2 + 0.00013 l^-4), l in um,
//     times the surface pressure ratio (Hansen, Travis 1974);
//   - E_j = B(l_j, T) / B(555 nm, T) (r0/r)^2 exp(-tau(l_j) m) above the horizon, else 0.
// The spectrum goes to the kernels through the scene's sun table (sdd_set_sun).
#include <cmath>
#include <string>
#include <vector>

#include "host.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kDeg = kPi / 180.0;

struct SunGeometry {
  double elevation, azimuth;  // degrees; azimuth clockwise from north
  double dist2;               // (r0 / r)^2
};

SunGeometry sun_geometry(const sdd_daylight& p) {
  const double g = 2.0 * kPi * (p.day_of_year - 1) / 365.0;
  const double c1 = std::cos(g), s1 = std::sin(g), c2 = std::cos(2 * g), s2 = std::sin(2 * g);
  const double c3 = std::cos(3 * g), s3 = std::sin(3 * g);
  const double decl = 0.006918 - 0.399912 * c1 + 0.070257 * s1 - 0.006758 * c2 + 0.000907 * s2 - 0.002697 * c3 +
                      0.00148 * s3;
  const double eot_min = 229.18 * (0.000075 + 0.001868 * c1 - 0.032077 * s1 - 0.014615 * c2 - 0.040849 * s2);
  SunGeometry out;
  out.dist2 = 1.000110 + 0.034221 * c1 + 0.001280 * s1 + 0.000719 * c2 + 0.000077 * s2;
  // true solar time in minutes -> hour angle (0 at solar noon, positive in the afternoon)
  const double tst = 60.0 * p.clock_hours + eot_min + 4.0 * p.longitude_deg - 60.0 * p.utc_offset_hours;
  const double ha = (tst / 4.0 - 180.0) * kDeg;
  const double lat = p.latitude_deg * kDeg;
  double se = std::sin(lat) * std::sin(decl) + std::cos(lat) * std::cos(decl) * std::cos(ha);
  se = std::fmax(-1.0, std::fmin(1.0, se));
  out.elevation = std::asin(se) / kDeg;
  // from south toward west, turned to compass azimuth
  const double az_s = std::atan2(std::sin(ha), std::cos(ha) * std::sin(lat) - std::tan(decl) * std::cos(lat));
  out.azimuth = std::fmod(az_s / kDeg + 180.0 + 360.0, 360.0);
  return out;
}

double planck_nm(double lambda_nm, double t) {
  const double h = 6.62607015e-34, c = 299792458.0, k = 1.380649e-23;
  const double l = lambda_nm * 1e-9;
  return 2.0 * h * c * c / (l * l * l * l * l) / std::expm1(h * c / (l * k * t));
}

std::string check(const sdd_daylight* p, int32_t n_bins, float lmin, float lmax) {
  if (!p) return "daylight parameters are null";
  if (p->day_of_year < 1 || p->day_of_year > 366) return "day_of_year must lie in 1..366";
  if (!(p->clock_hours >= 0.0f && p->clock_hours <= 24.0f)) return "clock_hours must lie in [0, 24]";
  if (!(std::fabs(p->utc_offset_hours) <= 14.0f)) return "utc_offset_hours must lie in [-14, 14]";
  if (!(std::fabs(p->latitude_deg) <= 90.0f)) return "latitude must lie in [-90, 90]";
  if (!(std::fabs(p->longitude_deg) <= 180.0f)) return "longitude must lie in [-180, 180]";
  if (!std::isfinite(p->scene_x_azimuth_deg)) return "scene_x_azimuth_deg must be finite";
  if (!(p->temperature_k >= 1000.0f && p->temperature_k <= 100000.0f)) return "temperature must lie in 1e3..1e5 K";
  if (!(p->pressure_ratio >= 0.0f && p->pressure_ratio <= 10.0f)) return "pressure_ratio must lie in [0, 10]";
  if (n_bins < 1 || n_bins > sdd::kMaxBins) return "n_bins must lie in 1..128";
  if (!(lmin > 0.0f) || !(lmax > lmin) || !std::isfinite(lmax)) return "need 0 < lambda_min < lambda_max";
  return "";
}

}  // namespace

extern "C" int sdd_daylight_sun(const sdd_daylight* p, int32_t n_bins, float lmin, float lmax, float dir_to_sun[3],
                                float* irradiance, sdd_daylight_info* info) {
  const std::string e = check(p, n_bins, lmin, lmax);
  if (!e.empty()) {
    sdd::set_thread_error(e);
    return SDD_ERR_INVALID_ARG;
  }
  if (!dir_to_sun || !irradiance) {
    sdd::set_thread_error("null output");
    return SDD_ERR_INVALID_ARG;
  }
  const SunGeometry g = sun_geometry(*p);
  const double el = g.elevation * kDeg, az = g.azimuth * kDeg, psi = p->scene_x_azimuth_deg * kDeg;
  const double east = std::cos(el) * std::sin(az), north = std::cos(el) * std::cos(az), up = std::sin(el);
  // scene frame: +x at compass azimuth psi, +y = z x x, +z up
  dir_to_sun[0] = (float)(east * std::sin(psi) + north * std::cos(psi));
  dir_to_sun[1] = (float)(-east * std::cos(psi) + north * std::sin(psi));
  dir_to_sun[2] = (float)up;
  double mass = INFINITY;
  if (g.elevation > 0.0) {
    const double z = 90.0 - g.elevation;
    mass = 1.0 / (std::cos(z * kDeg) + 0.50572 * std::pow(96.07995 - z, -1.6364));
  }
  const double b555 = planck_nm(555.0, p->temperature_k);
  for (int j = 0; j < n_bins; ++j) {
    const double lam = lmin + (j + 0.5) * ((double)lmax - lmin) / n_bins;
    const double um = lam * 1e-3, um2 = um * um, um4 = um2 * um2;
    const double tau = p->pressure_ratio * 0.008569 / um4 * (1.0 + 0.0113 / um2 + 0.00013 / um4);
    irradiance[j] = g.elevation > 0.0 ? (float)(planck_nm(lam, p->temperature_k) / b555 * g.dist2 *
                                                std::exp(-tau * mass))
                                      : 0.0f;
  }
  if (info) {
    info->elevation_deg = (float)g.elevation;
    info->azimuth_deg = (float)g.azimuth;
    info->air_mass = (float)mass;
    info->distance_factor = (float)g.dist2;
  }
  return SDD_OK;
}

extern "C" int sdd_set_daylight(sdd_ctx* c, sdd_scene* s, const sdd_daylight* p, sdd_daylight_info* info) {
  if (!c || !s) {
    sdd::set_thread_error("null argument");
    return SDD_ERR_INVALID_ARG;
  }
  std::vector<float> E((size_t)s->hdr.n_bins);
  float dir[3];
  const int rc = sdd_daylight_sun(p, s->hdr.n_bins, s->hdr.lambda_min_nm, s->hdr.lambda_max_nm, dir, E.data(), info);
  if (rc) {
    c->err = sdd::thread_error();
    return rc;
  }
  return sdd_set_sun(c, s, dir, E.data());
}
