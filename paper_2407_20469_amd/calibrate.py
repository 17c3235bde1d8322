"""Measured ceilings of the current GPU for roofline reporting.

    python -m paper_2407_20469_amd.calibrate

Runs the library's probes: a sustained FP64 FMA loop, the same work on the
FP64 matrix cores and a plain 4 GiB copy (three repetitions).  Prints one
JSON line with the two FP64 rates in TFLOP/s and the copy bandwidth (read +
write bytes over time) in GB/s.  Under
`rocprofv3 --pmc FETCH_SIZE` / `WRITE_SIZE` the copy dispatches give the
counter-to-bytes scale: each copy moves exactly COPY_BYTES each way.
"""

import ctypes
import json

COPY_BYTES = 4 << 30


def main():
    import torch
    from paper_2407_20469_amd import apic
    lib = apic.load_library()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    blocks, iters = 256 * 64, 2000
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    apic._check("apic_calib_fma64", lib.apic_calib_fma64(ctypes.c_void_p(out.data_ptr()), blocks, 10, st))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    apic._check("apic_calib_fma64", lib.apic_calib_fma64(ctypes.c_void_p(out.data_ptr()), blocks, iters, st))
    e1.record()
    torch.cuda.synchronize()
    res = {"fp64_fma_tflops": blocks * 256 * iters * 256 / e0.elapsed_time(e1) / 1e9}
    apic._check("apic_calib_mfma64", lib.apic_calib_mfma64(ctypes.c_void_p(out.data_ptr()), blocks, 10, st))
    e0.record()
    apic._check("apic_calib_mfma64", lib.apic_calib_mfma64(ctypes.c_void_p(out.data_ptr()), blocks, iters, st))
    e1.record()
    torch.cuda.synchronize()
    res["fp64_mfma_tflops"] = blocks * 4 * iters * 8 * 2048 / e0.elapsed_time(e1) / 1e9
    a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(3):
        e0.record()
        apic._check("apic_calib_copy", lib.apic_calib_copy(ctypes.c_void_p(a.data_ptr()),
                                                           ctypes.c_void_p(b.data_ptr()),
                                                           COPY_BYTES, st))
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2 * COPY_BYTES / e0.elapsed_time(e1) / 1e6)
    res["copy_GBps"] = best
    res["copy_bytes_each_way"] = COPY_BYTES
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
