"""Autotuner of the evaluation strategy.

For each case (n, m, precision, cells) every strategy the library offers is
timed on the GPU (HIP events around bz_collide_batch, the plan's own timing):
the chunked plain pencil passes with 2, 4, 8 or (up to 17) a third or half of the
passes per stage-A launch,
the same passes with the last transforms as DFT matrix products on the matrix
cores (FP32, n in {16, 32, 48}), and the fused kernel (FP32, n in {16, 24, 32}) with 1, 2, 4 or 8 direction
chunks per cell and, for n = 16, one or two LDS slices.  A strategy is kept
only if its output agrees with the plain FP64 path on the same batch
(relative L2 over the batch <= 2e-5 in FP32, <= 1e-12 in FP64); the fastest
kept strategy is written to a tune table that bz_plan_create reads (see
bz_set_tune_table in include/bz.h).  The table shipped beside the library,
tune_gfx950.txt, was written by

    python -m paper_2505_03360_amd.autotune --out paper_2505_03360_amd/tune_gfx950.txt

(serving sizes n in {16, 24, 32, 48}, m = 32, 16 to 4096 cells, spherical design).
"""
from __future__ import annotations

import argparse
import os

import paper_2505_03360_amd as bz


FUSED_SLICES = {16: (1, 2), 24: (1,), 32: (2,)}


GEMM_N = (16, 32, 48)


def plain_ks(m: int):
    """Directions per stage-A launch tried for the plain path: 2, 4, 8 and the
    sizes that split the m + 1 passes into three or two equal launch pairs."""
    m1 = m + 1
    return sorted({2, 4, 8} | {k for k in (-(-m1 // 3), -(-m1 // 2)) if 8 < k <= 17})


def candidates(n: int, m: int, precision: int):
    out = [(bz.BZ_XF_PLAIN, k, 0) for k in plain_ks(m)]
    if precision == bz.BZ_FP32 and n in GEMM_N:
        out += [(bz.BZ_XF_DFT_GEMM, k, 0) for k in (2, 4, 8)]
    if precision == bz.BZ_FP32 and n in FUSED_SLICES:
        for s in FUSED_SLICES[n]:
            for c in (1, 2, 4, 8):
                if c <= m + 1:
                    out.append((bz.BZ_XF_FUSED, c, s))
    return out


def tune_case(n: int, m: int, precision: int, cells: int, reps: int = 5, L: float = 8.0, seed: int = 0):
    """Return (best, rows): best = (transform, chunks, slices, us_per_cell)."""
    import torch

    import bz_inputs as gen
    f = torch.from_numpy(gen.bimaxwellian_batch(cells, n, L, seed=seed)).cuda()
    kw = dict(L=L, m=m, dir_kind=bz.BZ_DIRS_DESIGN)
    ref = bz.Collider(n, cells, precision=bz.BZ_FP64, transform=bz.BZ_XF_PLAIN, **kw)(f)
    torch.cuda.synchronize()
    tol = 2e-5 if precision == bz.BZ_FP32 else 1e-12
    rows = []
    for x, c, s in candidates(n, m, precision):
        col = bz.Collider(n, cells, precision=precision, transform=x, chunks=c, slices=s, **kw)
        out = col(f)
        torch.cuda.synchronize()
        err = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref))
        bz.bz_plan_set_timing(col.plan, True)
        for _ in range(reps):
            col(f, out=out)
        ms = bz.bz_plan_last_times(col.plan)[3]
        bz.bz_plan_set_timing(col.plan, False)
        rows.append({"transform": x, "chunks": c, "slices": s, "ms": ms, "err": err, "ok": err <= tol})
        col.close()
        del out
        torch.cuda.empty_cache()
    ok = [r for r in rows if r["ok"]]
    if not ok:
        raise RuntimeError(f"no strategy passed parity for n={n} m={m} cells={cells}")
    b = min(ok, key=lambda r: r["ms"])
    return (b["transform"], b["chunks"], b["slices"], 1e3 * b["ms"] / cells), rows


def write_table(path: str, entries):
    """entries: iterable of (n, m, precision, cells, transform, chunks, slices, us_per_cell)."""
    with open(path, "w") as fh:
        fh.write("# arch n m precision max_cells transform chunks slices us_per_cell\n")
        for e in entries:
            fh.write("gfx950 %d %d %d %d %d %d %d %.4f\n" % tuple(e))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[16, 24, 32, 48])
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--cells", type=int, nargs="+", default=[16, 64, 128, 256, 512, 1024, 4096])
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--out", default=os.path.join(os.getcwd(), "tune_table.txt"))
    args = ap.parse_args()
    prec = bz.BZ_FP32 if args.precision == "fp32" else bz.BZ_FP64
    entries = []
    for n in args.n:
        for cells in args.cells:
            best, rows = tune_case(n, args.m, prec, cells)
            for r in rows:
                print(f"n={n} cells={cells} transform={r['transform']} chunks={r['chunks']} "
                      f"slices={r['slices']} {r['ms']:.4f} ms err={r['err']:.2e} {'ok' if r['ok'] else 'REJECTED'}",
                      flush=True)
            entries.append((n, args.m, prec, cells) + best)
    write_table(args.out, entries)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
