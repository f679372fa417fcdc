"""Plain device copy of a known size (1 GiB, three times).

Run under rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE): what the counters
report for these copies scales the counters of the sort's kernels into HBM
bytes (the factors are recorded in profiles/hbm_traffic.json)."""
import torch

N = 1 << 30

if __name__ == "__main__":
    a = torch.empty(N, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x %d bytes" % N, flush=True)
