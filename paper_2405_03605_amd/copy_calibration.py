"""Plain device copy of known size, used to scale rocprofv3's FETCH_SIZE and
WRITE_SIZE counters into HBM bytes: the counters of this run are compared with
the 1 GiB read and 1 GiB written that the copy must move.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2405_03605_amd.copy_calibration
"""
import torch

BYTES = 1 << 30


def main():
    a = torch.ones(BYTES // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {BYTES} bytes", flush=True)


if __name__ == "__main__":
    main()
