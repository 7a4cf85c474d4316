"""Launch autotuner for the buffer kernels and the batch split step.

For every operation (ECB encrypt, ECB decrypt, CTR), key size and buffer
size bucket it times every candidate launch configuration (table layout,
blocks per thread -- i.e. blocks per wave step = 64 x blocks_per_thread --,
workgroup size, or the bitsliced kernel) with HIP events on the current
stream, keeps the fastest, and installs the result in the library with
aes_set_tuned.  For batches it times the split granularity (the block
multiple on which a wave's share of a message starts and ends) on a ragged
multi-message workload.  Every candidate is timed per launch with HIP
events and scored by its median launch.  The table (the winning entries
and the batch split, keyed by the GPU's architecture and compute-unit
count) is saved as JSON; the binding installs the committed table for
gfx950 when it is imported.  The raw sweep goes to a separate file
(--log), not into the table.

    python -m paper_1403_7295_amd.autotune --out paper_1403_7295_amd/tuned_gfx950.json --log sweep.json
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuned_gfx950.json")

# table layouts: 0 four tables x 32 copies, 1 two x 64, 3 one x 64 with
# rotations (two workgroups per compute unit), 4 four unreplicated tables
TABLE_CANDIDATES = [dict(layout=l, blocks_per_thread=b, wg_size=w, grid=0)
                    for l in (0, 1, 3, 4) for b in (1, 2, 4) for w in (256, 512, 1024)]
BITSLICED = dict(layout=2, blocks_per_thread=0, wg_size=0, grid=0)
# (label, mode, decrypt)
OPS = (("ecb_enc", "ecb", 0), ("ecb_dec", "ecb", 1), ("ctr", "ctr", 0))
# size buckets: the size tuned at, and the smallest size the result applies to
BUCKETS = ((1 << 16, 0), (1 << 20, 1 << 18), (1 << 24, 1 << 22), (1 << 30, 1 << 27))
SPLIT_CANDIDATES = (128, 256, 512, 1024)
BATCH_BPT_CANDIDATES = (2, 4)


def _time(torch, fn, reps, warm=2):
    """Median launch time in seconds over `reps` launches, each between its
    own pair of HIP events (after `warm` untimed ones)."""
    s = torch.cuda.current_stream()
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(s)
        fn()
        b.record(s)
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) / 1e3 for a, b in evs)
    return t[len(t) // 2]


def tune_plain(A, torch, nrs=(10, 12, 14), buckets=BUCKETS, verbose=False):
    """Returns (entries for aes_set_tuned, measurements)."""
    import seedgen
    big = max(sz for sz, _ in buckets)
    x = seedgen.data_torch(77, 0, big, "cuda")
    y = torch.empty_like(x)
    ctr0 = seedgen.nonce(77, 0)
    entries, log = [], []
    A.aes_set_tuned([])
    try:
        for nr in nrs:
            rk, _ = A.aes_expand_key(seedgen.key(77, nr, {10: 128, 12: 192, 14: 256}[nr]))
            for label, mode, dec in OPS:
                fn = A.aes_decrypt if dec else A.aes_encrypt
                cands = TABLE_CANDIDATES + ([] if (mode == "ecb" and dec) else [BITSLICED])
                for size, min_bytes in buckets:
                    reps = max(7, min(200, (1 << 28) // size))
                    best = None
                    for cfg in cands:
                        A.aes_set_launch(cfg)
                        t = _time(torch, lambda: fn(x, y, size, rk, nr, mode, ctr0=ctr0), reps)
                        log.append(dict(op=label, Nr=nr, bytes=size, cfg=cfg, seconds=t,
                                        GBps=size / t / 1e9))
                        if best is None or t < best[0]:
                            best = (t, cfg)
                    A.aes_set_launch(None)
                    entries.append(dict(mode=mode, decrypt=dec, Nr=nr, min_bytes=min_bytes,
                                        cfg=best[1], tuned_at_bytes=size,
                                        GBps=round(size / best[0] / 1e9, 1)))
                    if verbose:
                        print("%s Nr=%d %10d B: %s %.1f GB/s" % (label, nr, size, best[1],
                                                                  size / best[0] / 1e9), flush=True)
    finally:
        A.aes_set_launch(None)
    return entries, log


def tune_batch(A, torch, nmsg=2000, verbose=False):
    """Best split granularity and blocks per thread of the batch kernels
    (their table layout is the buffer kernels' four tables x 32 copies,
    which the plain sweep finds fastest for every operation) on the ragged
    multi-message workload (a 2,000-message slice of it) and on 4 KiB
    sectors (8,192 messages), scored by the sum of the two times."""
    import seedgen
    lens, keybits, keys, _ = seedgen.ragged_batch(4, nmsg)
    work = [(A.make_descs(lens, keybits=keybits, mode="ecb"), keys, int(lens.sum()))]
    nsec = 8192
    skeys = np.zeros((nsec, 32), np.uint8)
    skeys[:, :16] = np.random.default_rng(6).integers(0, 256, (nsec, 16), dtype=np.uint8)
    work.append((A.make_descs(np.full(nsec, 4096), keybits=128, mode="ctr", ctr0=np.zeros(16, np.uint8)), skeys,
                 nsec * 4096))
    x = seedgen.data_torch(4, 0, max(t for _, _, t in work), "cuda")
    y = torch.empty_like(x)
    results = []
    for bpt in BATCH_BPT_CANDIDATES:
        for split in SPLIT_CANDIDATES:
            secs = []
            for descs, k, total in work:
                b = A.Batch(descs, k, x, y, tile_blocks=split, blocks_per_thread=bpt)
                secs.append(_time(torch, lambda: b.launch_graph(), 7))
                b.close()
            results.append(dict(tile_blocks=split, blocks_per_thread=bpt, seconds=sum(secs),
                                ragged_GBps=work[0][2] / secs[0] / 1e9, sectors_GBps=work[1][2] / secs[1] / 1e9))
            if verbose:
                print("batch split %5d bpt %d: ragged %.1f GB/s, 4 KiB sectors %.1f GB/s"
                      % (split, bpt, results[-1]["ragged_GBps"], results[-1]["sectors_GBps"]), flush=True)
    best = min(results, key=lambda r: r["seconds"])
    return best["tile_blocks"], best["blocks_per_thread"], results


def device_key(torch):
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return "%s_%dcu" % (arch, p.multi_processor_count)


def save(path, table):
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def load(path=DEFAULT_TABLE):
    with open(path) as f:
        return json.load(f)


def apply(A, table):
    """Install a saved table's launch entries in the library."""
    A.aes_set_tuned([dict(mode=e["mode"], decrypt=e["decrypt"], Nr=e["Nr"], min_bytes=e["min_bytes"],
                          cfg=e["cfg"]) for e in table["entries"]])


def main():
    ap = argparse.ArgumentParser(description="tune launch configurations on this GPU")
    ap.add_argument("--out", default=None)
    ap.add_argument("--log", default=None, help="where to write every measurement of the sweep")
    ap.add_argument("--nr", type=int, nargs="*", default=[10, 12, 14])
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="re-tune only the batch split of the committed table; write it to --out "
                         "(default: in place)")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    from paper_1403_7295_amd import aesgpu as A
    t0 = time.time()
    if args.batch_only:
        table = load(DEFAULT_TABLE)
        table["batch_tile_blocks"], table["batch_blocks_per_thread"], blog = tune_batch(A, torch, verbose=True)
        save(args.out or DEFAULT_TABLE, table)
        if args.log:
            save(args.log, {"batch": blog})
        print("batch_tile_blocks", table["batch_tile_blocks"], "batch_blocks_per_thread",
              table["batch_blocks_per_thread"])
        return
    entries, log = tune_plain(A, torch, tuple(args.nr), verbose=True)
    table = {"device": device_key(torch), "entries": entries}
    sweep = {"plain": log}
    if not args.no_batch:
        split, bpt, blog = tune_batch(A, torch, verbose=True)
        table["batch_tile_blocks"] = split
        table["batch_blocks_per_thread"] = bpt
        sweep["batch"] = blog
    table["seconds"] = round(time.time() - t0, 1)
    if args.out:
        save(args.out, table)
    if args.log:
        save(args.log, sweep)
    print(json.dumps(table, indent=1))


if __name__ == "__main__":
    main()
