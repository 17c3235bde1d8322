// Host-only driver for the geometry plan builder, built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_plan_sanitize.py: builds the
// plans of every tile size and LED count the workloads use (plus rejected
// geometries) and walks every table, so out-of-range writes or reads,
// signed overflow and similar faults in the builder abort the run.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2407_20469_amd/csrc/plan.hpp"

namespace {

std::vector<int32_t> ring(int n, double na_ill, int count, double offset, bool inward) {
  const double rho = na_ill * n * 0.4 / 0.52, r = 0.25 * n * 0.4 / 0.52;
  std::vector<int32_t> out;
  for (int i = 0; i < count; ++i) {
    const double a = 2.0 * M_PI * (i + offset) / count;
    int bx = 0, by = 0;
    double best = 1e300;
    for (int x = (int)std::floor(rho * std::cos(a)) - 2; x <= (int)std::ceil(rho * std::cos(a)) + 2; ++x)
      for (int y = (int)std::floor(rho * std::sin(a)) - 2; y <= (int)std::ceil(rho * std::sin(a)) + 2; ++y) {
        if (inward && x * x + y * y > r * r) continue;
        const double d = std::hypot(x - rho * std::cos(a), y - rho * std::sin(a));
        if (d < best) best = d, bx = x, by = y;
      }
    out.push_back(bx);
    out.push_back(by);
  }
  return out;
}

long walk(const apic::GeomPlan &p) {
  long s = p.n_rows + p.n_pix + (long)p.coords.size() + (long)p.masks.size();
  for (uint32_t v : p.row_il) s += v & 0xff;
  for (uint32_t v : p.pix_tab) s += v & 1;
  for (int16_t v : p.known_at) s += v < 0;
  for (const apic::DfStep &d : p.steps) {
    s += d.nu + d.m + d.ne;
    for (int64_t k = 0; k < d.nu; ++k) s += p.coords[d.off_u + k] & 1;
    for (int64_t k = 0; k < d.ne; ++k) s += p.coords[d.off_e + k] & 1;
  }
  return s + p.lay.stride;
}

}  // namespace

int main() {
  int built = 0, rejected = 0;
  for (int n : {64, 128, 256, 512})
    for (int nbf : {8, 12, 16}) {
      for (bool dark : {true, false}) {
        if (n == 512 && (nbf != 16 || !dark)) continue;  // one 512 px plan keeps the run short
        std::vector<int32_t> kbf = ring(n, 0.25, nbf, 0.0, true), kdf;
        if (dark) {
          kdf = ring(n, 0.30, nbf, 0.0, false);
          std::vector<int32_t> k2 = ring(n, 0.38, nbf, 0.5, false);
          kdf.insert(kdf.end(), k2.begin(), k2.end());
        }
        apic_geometry g{};
        g.n = n;
        g.upsample = n <= 512 ? 2 : 1;
        g.dx_um = 0.4;
        g.wavelength_um = 0.52;
        g.na_obj = 0.25;
        g.n_bf = nbf;
        g.n_df = (int)kdf.size() / 2;
        g.k_bf = kbf.data();
        g.k_df = kdf.empty() ? nullptr : kdf.data();
        g.ridge_pupil = 1e-9;
        g.ridge_darkfield = 1e-4;
        g.log_floor_rel = 1e-6;
        g.pupil_bands = 1;
        apic::GeomPlan p;
        const apic_status rc = apic::build_geom_plan(g, p);
        if (rc == APIC_OK) {
          ++built;
          std::printf("n %d n_bf %d n_df %d rows %d bands %zu pix %d steps %zu walk %ld\n", n, nbf,
                      g.n_df, p.n_rows, p.band_rows.size(), p.n_pix, p.steps.size(), walk(p));
        } else {
          ++rejected;
        }
      }
    }
  // a geometry whose darkfield shift would wrap must be rejected, not built
  std::vector<int32_t> kbf = ring(64, 0.25, 8, 0.0, true), kdf = ring(64, 0.9, 8, 0.0, false);
  apic_geometry g{64, 2, 0.4, 0.52, 0.25, 8, 8, kbf.data(), kdf.data(), 1e-9, 1e-4, 1e-6};
  apic::GeomPlan p;
  if (apic::build_geom_plan(g, p) == APIC_OK) {
    std::printf("wrapping geometry was accepted\n");
    return 1;
  }
  std::printf("built %d rejected %d\n", built, rejected);
  return built >= 15 ? 0 : 1;
}
