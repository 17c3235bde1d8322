"""Illumination vectors on the DFT lattice.

The paper's LEDs sit on rings (12 NA-matched on one ring, 22 darkfield on two
outer rings, Sec. 3) but the reconstruction needs each illumination vector as a
point of the discrete frequency grid (Sec. 2.3 speaks of the "flattened
position" of k_n).  Rule used here:

* a ring of n LEDs at illumination NA ``na_ill`` has radius
  rho = na_ill * N * dx / lambda bins and azimuths 2 pi (i + o) / n;
* each LED is the lattice point (kx, ky) nearest to rho (cos a, sin a);
* NA-matched LEDs are restricted to |k| <= r (pupil radius), so the DC of the
  shifted spectrum stays inside the pupil;
* ties go to the larger |k|, then the smaller angular error, then the larger
  kx, then the larger ky.
"""

import math


def _angle_err(x, y, a):
    d = math.atan2(y, x) - a
    return abs(math.atan2(math.sin(d), math.cos(d)))


def led_ring(n, na_ill, count, offset=0.0, inward=False, dx_um=0.4, wavelength_um=0.52,
             na_obj=0.25):
    """Integer (kx, ky) illumination vectors of one ring, in azimuth order."""
    rho = na_ill * n * dx_um / wavelength_um
    r = na_obj * n * dx_um / wavelength_um
    out = []
    for i in range(count):
        a = 2.0 * math.pi * (i + offset) / count
        tx, ty = rho * math.cos(a), rho * math.sin(a)
        best = None
        for x in range(math.floor(tx) - 2, math.ceil(tx) + 3):
            for y in range(math.floor(ty) - 2, math.ceil(ty) + 3):
                if inward and x * x + y * y > r * r:
                    continue
                key = (round((x - tx) ** 2 + (y - ty) ** 2, 9), -(x * x + y * y),
                       round(_angle_err(x, y, a), 9), -x, -y)
                if best is None or key < best[0]:
                    best = (key, (x, y))
        out.append(best[1])
    return out


def led_rings(n, rings, dx_um=0.4, wavelength_um=0.52, na_obj=0.25):
    """Concatenate several rings given as (na_ill, count, offset, inward) tuples."""
    out = []
    for na_ill, count, offset, inward in rings:
        out += led_ring(n, na_ill, count, offset, inward, dx_um, wavelength_um, na_obj)
    return out
