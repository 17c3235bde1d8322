"""Three-wavelength stained-slide workload on the GPU (Sec. 3.3: the method
runs per colour channel, then the amplitudes are combined and white
balanced).

Three 128 px tiles, each imaged at 0.63, 0.52 and 0.47 um (pupil radius and
LED lattice scale with 1/lambda; per-channel pupils with a chromatic
defocus), run as one prepared batch of three geometry classes.  Bars: each
channel's first tile against the FP64 oracle at field rel-L2 1e-4 and Noll
coefficients 1e-3 rad; the colour image and grey-world gains against the
oracle's combination of the same GPU fields at 1e-6 relative (FP32 amplitudes,
FP64 channel means).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from apic_synth.rgb import config_rgb
from oracle import rgb as orgb
from paper_2407_20469_amd import apic
from gpu_helpers import oracle_geometry, rel_l2, workload_images

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _log(msg):
    print(f"[gpu-test] {msg}", flush=True)


def test_rgb_channels_and_colour_image():
    T = 3
    ws = config_rgb(n_tiles=T, n=128)
    imgs = [workload_images(w, photons=1e4) for w in ws]
    plan = apic.Plan([w.geometry_kwargs() for w in ws])
    order = [c for t in range(T) for c in range(3)]          # tile-major, R G B
    descs, n_img_el, n_fld_el = apic.mixed_descs(plan, order)
    flat = np.concatenate([imgs[c][t].ravel() for t in range(T) for c in range(3)])
    images = torch.tensor(flat.astype(np.float32), device=DEV)
    field = torch.empty(n_fld_el, dtype=torch.complex64, device=DEV)
    zern = torch.empty((3 * T, 15), dtype=torch.float32, device=DEV)
    status = torch.empty((3 * T,), dtype=torch.int32, device=DEV)
    batch = apic.Batch(plan, descs)
    _log(f"batch of {3 * T} tiles over three wavelengths")
    batch.reconstruct(images, field, zern, status, apic.Workspace())
    torch.cuda.synchronize()
    nf = 256
    f = field.view(3 * T, nf, nf)
    z = zern.cpu().numpy()
    for c, w in enumerate(ws):
        ref = oracle.reconstruct(imgs[c][0].astype(np.float64), oracle_geometry(w))
        err = rel_l2(f[c].cpu().numpy(), ref["field"])
        dz = np.abs(z[c] - ref["c"]).max()
        _log(f"channel {w.extra['channel']} (r = {w.r:.2f}): field rel-L2 {err:.2e}, "
             f"max|dc| {dz:.1e}, c4 {z[c][3]:+.3f} (true {w.coeffs[0][3]:+.3f})")
        assert err < 1e-4 and dz < 1e-3
    # chromatic defocus: the estimated Z4 differences follow the true ones
    d_est = z[0][3] - z[2][3]
    d_true = ws[0].coeffs[0][3] - ws[2].coeffs[0][3]
    _log(f"Z4(R) - Z4(B): estimated {d_est:+.3f}, true {d_true:+.3f}")
    assert abs(d_est - d_true) < 0.05
    chans = [f[c::3].contiguous() for c in range(3)]
    img, g = apic.rgb_combine(*chans)
    ref_img, ref_g = orgb.combine([x.cpu().numpy() for x in chans])
    e_img = np.abs(img.cpu().numpy() - ref_img).max() / ref_img.max()
    _log(f"grey-world gains {g} vs {ref_g}; colour image max rel err {e_img:.2e}")
    assert np.allclose(g, ref_g, rtol=1e-6) and e_img < 1e-6
    img2, g2 = apic.rgb_combine(*chans, gains=(1.0, 2.0, 0.5))
    ref2, _ = orgb.combine([x.cpu().numpy() for x in chans], (1.0, 2.0, 0.5))
    assert np.array_equal(g2, np.float32([1.0, 2.0, 0.5]))
    assert np.abs(img2.cpu().numpy() - ref2).max() / ref2.max() < 1e-6
