"""Reference copy for HBM traffic counters: three copies of 256 MiB of FP64.

Run under ``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``; the ratio of
the known bytes to what each counter reports for the copy kernel scales the
same counters of the library's kernels (bytes moved to and from HBM).
"""
import torch


def main():
    n = 32 * 1024 * 1024  # 256 MiB of float64
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied 3 x 256 MiB", flush=True)


if __name__ == "__main__":
    main()
