"""Copy-kernel calibration for the HBM byte counters.

Runs a plain device-to-device copy of a known size (1 GiB read + 1 GiB
written, far above the caches) a few times.  Under a counter profiler the
FETCH_SIZE / WRITE_SIZE readings of this kernel, divided by the known bytes,
give the factor that turns the counter readings of the search kernels into
bytes.

    python -m paper_1810_09898_amd.calib
"""
import torch


def main(nbytes=1 << 30, reps=3):
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy calibration: {reps} copies of {nbytes} bytes", flush=True)


if __name__ == "__main__":
    main()
