"""One whole weighted-quadrature step on a seeded mesh, plus a plain device copy of known
size, as a short program for hardware-counter collection:

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2605_29334_amd.profile_run
    rocprofv3 --pmc WRITE_SIZE -- python3 -m paper_2605_29334_amd.profile_run

The copy (an elementwise kernel b = a * 1 over --copy-mib MiB of doubles) calibrates the
counters: its true HBM traffic is known (read a once, write b once), so counter bytes
of the WQ kernels are scaled by copy bytes / counter bytes of the copy.
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--density", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=2000)
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()

    import torch
    import fixtures as fx
    import paper_2605_29334_amd.wq as W

    torch.cuda.set_device(0)
    F = fx.fixture_eps(args.N, args.density, (3, 5, 6), displace=0.05, seed=args.seed)
    mesh = W.Mesh(F)
    stream = torch.cuda.current_stream()
    pts = W.Points(mesh, stream=stream)
    x = pts.get(W.ARR_X).reshape(-1, 2)
    c = (1 + 0.5 * torch.sin(2 * torch.pi * x[:, 0]) * torch.sin(2 * torch.pi * x[:, 1])).contiguous()
    k = (1 + 0.5 * torch.cos(torch.pi * x[:, 0]) * torch.cos(torch.pi * x[:, 1])).contiguous()
    wts = W.Weights(mesh, pts, W.WQ_FAM_MASS | W.WQ_FAM_DX | W.WQ_FAM_DY, tau=1e-12, stream=stream)
    W.assemble_mass_stiffness(pts, wts, c, k, stream=stream)
    torch.cuda.synchronize()
    n = args.copy_mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(f"[profile_run] N={args.N} rows={pts.n_rows} nnz={pts.nnz} copy_bytes={8 * n}", flush=True)


if __name__ == "__main__":
    main()
