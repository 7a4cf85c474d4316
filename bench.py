#!/usr/bin/env python3
"""Throughput benchmark: AES-128 ECB encryption of a 1 GiB device-resident
buffer on one MI355X, through the C ABI (aes_expand_key + aes_encrypt).

One step = Key Expansion on the host + one ECB encryption of the whole 1 GiB
buffer (67,108,864 16-byte blocks) of seeded uniform random bytes.  The
input is produced on the device before the timed region.  W untimed steps,
then exactly K timed steps between two synchronisations; every launch is
also bracketed by HIP events on the stream it runs on, which gives the
kernel's own duration for the roofline figures.

Prints one JSON line.  Besides the headline it carries:
  roofline      the binding ceiling (LDS-lookup issue rate or HBM), with the
                algorithmic work of one launch divided by its measured time;
  roofline_hbm, roofline_issue   both ceilings (the HBM one also against the
                copy kernel's measured bandwidth);
  cpu_baseline  the oracle (plain byte-oriented C AES) on the host's cores,
                run with the paper's pthreads chunking on a bounded sample;
  cpu_context   for comparison only: `openssl speed` (AES-NI) on the same cores;
  secondary     the other operations of the path on the same buffer (CTR,
                ECB decryption, AES-256) and the copy kernel's bandwidth.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import seedgen  # noqa: E402

GiB = 1 << 30
HBM_PEAK_GBS = 8000.0             # MI355X HBM3E, published
CUS, CLOCK_GHZ = 256, 2.4          # MI355X compute units, peak engine clock
LDS_LANES_PER_CLK = 32             # LDS: 32 banks x 4 B per clock per CU
LDS_PEAK_TLOOKUPS = CUS * CLOCK_GHZ * 1e9 * LDS_LANES_PER_CLK / 1e12   # 19.66
# warm-up launches of each 1 GiB secondary measurement (≈ 10 ms): after a
# pause on the host side the first launches run slower (GCM encryption, the
# first measured after the XTS legs' set-up, came out 10 % below decryption
# with two)
SEC_WARMUP = 10
KERNEL_SRC = os.path.join(ROOT, "paper_1403_7295_amd", "csrc", "aes_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cipher_kernel_aes128_ecb_enc_1GiB.json")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nbytes", type=int, default=GiB)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--cpu-sample-mib", type=int, default=32)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--served-requests", type=int, default=20000)
    return ap.parse_args()


def lookups_per_block(nr, ctr=False):
    # 16 table lookups per round; CTR saves 12 of round 1's (shared nonce columns)
    return 16 * nr - (12 if ctr else 0)


def launch_stats(times):
    """Per-launch kernel times (seconds): mean, median, min, max, and the
    paper's style of average (Section V drops runs that deviate much; read
    here as dropping those beyond median +- 2 MAD), in microseconds."""
    t = sorted(times)
    med = t[len(t) // 2]
    mad = sorted(abs(x - med) for x in t)[len(t) // 2]
    kept = [x for x in t if abs(x - med) <= 2 * mad] or t
    us = lambda v: round(v * 1e6, 2)  # noqa: E731
    return {"mean": us(sum(t) / len(t)), "median": us(med), "min": us(t[0]), "max": us(t[-1]),
            "paper_style_mean": us(sum(kept) / len(kept)), "launches": len(t), "kept": len(kept)}


def timed_launches(torch, stream, launch, steps, warmup, median=False, stats=None):
    """Runs `launch` warmup + steps times; returns (wall seconds of the timed
    steps, mean kernel seconds from HIP events on `stream`; the median
    instead with median=True).  `stats`, a dict, receives launch_stats()."""
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        launch()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = sorted(a.elapsed_time(b) / 1e3 for a, b in evs)
    kern = times[len(times) // 2] if median else sum(times) / steps
    if stats is not None:
        stats.update(launch_stats(times))
    return wall, kern


def kernel_source_sha():
    """Hash of the device code of the buffer kernels."""
    h = hashlib.sha256()
    for name in ("aes_kernels.hip", "cipher_core.h"):
        with open(os.path.join(os.path.dirname(KERNEL_SRC), name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(launch):
    """HBM bytes per launch from committed hardware-counter runs, if they were
    taken on the kernel source and launch configuration in use now; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_sha() or t.get("launch") != launch:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_runs(o, rk, nr, x, threads, reps=5):
    """One warm-up run, then `reps` timed runs of the oracle's pthreads
    method (seconds from thread creation to the last join, CLOCK_MONOTONIC
    inside the oracle): the median, and the mean after dropping runs beyond
    median +- 2 MAD (the paper's style, Section V)."""
    o.par_run(0, rk, nr, x, threads)
    t = sorted(o.par_run(0, rk, nr, x, threads)[1] for _ in range(reps))
    med = t[len(t) // 2]
    mad = sorted(abs(v - med) for v in t)[len(t) // 2]
    kept = [v for v in t if abs(v - med) <= 2 * mad] or t
    return med, sum(kept) / len(kept), t


def cpu_baseline(sample_bytes):
    """The oracle, untuned, on all host cores with the paper's pthreads split,
    and on one thread for the per-core figure (the paper's Table I reports
    both).  A bounded sample of the headline workload: the oracle runs at
    tens of MB/s, so the whole 1 GiB would take about a quarter of a minute
    per repetition on all cores and several minutes on one."""
    from oracle import ref
    o = ref.default()
    key = seedgen.key(2, 0, 128)
    rk, nr = o.expand_key(key)
    x = seedgen.data_np(2, 0, sample_bytes)
    threads = len(os.sched_getaffinity(0))
    med, paper, _ = oracle_runs(o, rk, nr, x, threads)
    # one thread on an eighth of the sample
    one_bytes = max(sample_bytes // 8, 1 << 20)
    one_med, one_paper, _ = oracle_runs(o, rk, nr, x[:one_bytes], 1)
    return {"value": round(sample_bytes / med / 1e9, 5), "unit": "GB/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "AES-128 ECB encrypt of the first %d MiB of the headline workload's seeded input "
                      "(1 GiB would take ~%.0f s per run), %d pthreads over contiguous whole-block chunks; "
                      "1 warm-up + median of 5 runs, %.2f s each"
                      % (sample_bytes >> 20, med * (1 << 30) / sample_bytes, threads, med),
            "paper_style_GB/s": round(sample_bytes / paper / 1e9, 5),
            "single_thread_GB/s": round(one_bytes / one_med / 1e9, 5),
            "single_thread_paper_style_GB/s": round(one_bytes / one_paper / 1e9, 5),
            "single_thread_sample": "the first %d MiB, 1 thread, 1 warm-up + median of 5 runs, %.2f s each"
                                    % (one_bytes >> 20, one_med)}


def cpu_context_openssl(seconds=1, block=16384):
    """An optimised CPU for context, beside the oracle: `openssl speed` of
    AES-128 ECB through EVP (AES-NI where the host has it) in one process per
    host core, 16 KiB blocks.  A comparison system, not the oracle and not a
    target; None when the executable is missing or does not answer."""
    import shutil
    import subprocess
    exe = shutil.which("openssl")
    if exe is None:
        return None
    procs = len(os.sched_getaffinity(0))
    cmd = [exe, "speed", "-evp", "aes-128-ecb", "-seconds", str(seconds), "-bytes", str(block),
           "-multi", str(procs)]
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=60)
    except (OSError, subprocess.TimeoutExpired):
        return None
    rate = None
    for line in r.stdout.splitlines():
        f = line.split()
        if len(f) == 2 and f[0] == "evp" and f[1].endswith("k"):
            rate = float(f[1][:-1]) * 1000.0   # bytes per second, all processes
    if r.returncode != 0 or rate is None:
        return None
    return {"GB/s": round(rate / 1e9, 2), "processes": procs, "kind": "openssl speed (comparison system)",
            "cpu_model": cpu_model(), "command": " ".join(["openssl"] + cmd[1:])}


LDS_GATHER_ROUNDS = 4096


def leg(torch, stream, launch, nbytes, reps=10, warmup=None):
    """One secondary measurement: `reps` launches after `warmup` untimed
    ones (SEC_WARMUP by default), each timed with HIP events on `stream`;
    GB/s of `nbytes` over the median launch, beside every launch statistic
    (one slow launch moves the mean, not the median)."""
    st = {}
    timed_launches(torch, stream, launch, reps, SEC_WARMUP if warmup is None else warmup, stats=st)
    return {"GB/s": round(nbytes / (st["median"] * 1e-6) / 1e9, 1), "launch_us": st}


def bench_lds_gather(torch, A, dev, stream, rounds=LDS_GATHER_ROUNDS, steps=20, warmup=3, layout=0):
    """The LDS calibration kernel in the cipher's launch shape: the 32-bit,
    own-bank lookups per second the LDS accepts with no global memory traffic
    and the cipher's VALU cost per lookup, and the rate of the cycle counter
    its waves read (s_memtime over the constant-rate s_memrealtime).  Layout
    0: the cipher's four tables x 32 copies, one workgroup per compute unit;
    layout 3: one table x 64 copies, two."""
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    waves = cus * 16 * 2     # room for two workgroups of 16 waves per compute unit
    rec = torch.zeros(waves * 3, dtype=torch.int64, device=dev)
    got = {}

    def launch():
        got["waves"], got["khz"] = A.aes_lds_gather(rec, rounds, stream=stream, layout=layout)

    _, k = timed_launches(torch, stream, launch, steps, warmup)
    w = got["waves"]
    lookups = w * 64 * 16 * rounds
    r = rec.view(-1, 3)[:w].cpu().double()
    cycles, ticks = float(r[:, 0].mean()), float(r[:, 1].mean())
    clock = cycles / (ticks / (got["khz"] * 1e3)) / 1e9 if ticks > 0 and got["khz"] > 0 else None
    if clock is not None and not 0.5 < clock < 3.5:
        clock = None    # the cycle counter does not count engine clocks here
    rate = lookups / k / 1e12
    out = {"Tlookup/s": round(rate, 3), "kernel_us": round(k * 1e6, 1), "lookups_per_launch": lookups,
           "waves": w, "layout": layout, "counter_clock_GHz": round(clock, 3) if clock else None}
    if clock:
        out["lookups_per_counter_clk_per_cu"] = round(rate * 1e12 / cus / (clock * 1e9), 2)
    return out


def bench_size_sweep(torch, A, dev, stream, sizes=(1 << 20, 1 << 22, 1 << 24, 1 << 26, 1 << 28, 1 << 30, 1 << 32)):
    """AES-256 ECB and CTR encryption of buffers of seeded random bytes from
    1 MiB to 4 GiB in steps of 4x (16 MiB, 256 MiB and 4 GiB are the named
    points), as the paper sweeps file size: GB/s per size.  Buffers up to
    16 MiB stay in the caches between repetitions."""
    key = seedgen.key(3, 0, 256)
    ctr0 = seedgen.nonce(3, 0)
    rk, nr = A.aes_expand_key(key)
    x = seedgen.data_torch(3, 0, max(sizes), dev)
    y = torch.empty_like(x)
    rows = []
    for n in sizes:
        for mode in ("ecb", "ctr"):
            reps = max(5, min(200, (1 << 31) // n))
            row = leg(torch, stream, lambda: A.aes_encrypt(x, y, n, rk, nr, mode, ctr0=ctr0, stream=stream),
                      n, reps, 3)
            rows.append(dict({"bytes": n, "mode": mode}, **row, cache_resident=n <= (1 << 24),
                             launch=A.aes_get_launch(n, mode, False, nr)))
    del x, y
    torch.cuda.empty_cache()
    return {"workload": "AES-256 encrypt, ECB and CTR, 1 MiB .. 4 GiB in steps of 4x",
            "statistic": "median launch time (HIP events) over the repetitions", "points": rows}


def bench_batched(torch, A, dev, stream, reps=5):
    """The ragged multi-message workload: 10,000 messages, lengths
    log-uniform in [16 B, 16 MiB], half AES-128 and half AES-256 keys, ECB
    encrypt.  One graph launch (on-device key expansion, the plan, persistent
    kernels) against one aes_expand_key + aes_encrypt per message."""
    lens, keybits, keys, _ = seedgen.ragged_batch(4, 10000)
    descs = A.make_descs(lens, keybits=keybits, mode="ecb")
    total = int(lens.sum())
    x = seedgen.data_torch(4, 0, total, dev)
    y = torch.empty_like(x)
    b = A.Batch(descs, keys, x, y)
    wall, kern = timed_launches(torch, stream, lambda: b.launch_graph(stream), reps, 2)
    offs = [int(o) for o in descs["in_off"]]
    sizes = [int(n) for n in lens]
    kl = [keys[m][:keybits[m] // 8] for m in range(len(lens))]

    def per_message():
        for o, n, k in zip(offs, sizes, kl):
            rk, nr = A.aes_expand_key(k)
            A.aes_encrypt(x[o:o + n], y[o:o + n], n, rk, nr, A.AES_MODE_ECB, stream=stream)

    pwall, _ = timed_launches(torch, stream, per_message, 2, 1)
    b.close()
    del x, y
    torch.cuda.empty_cache()
    return {"workload": "10,000 messages, log-uniform 16 B..16 MiB, AES-128/256 50/50, ECB encrypt",
            "bytes": total,
            "batched_graph_GB/s": round(total * reps / wall / 1e9, 1),
            "batched_graph_ms": round(wall / reps * 1e3, 3),
            "plain_per_message_GB/s": round(total * 2 / pwall / 1e9, 1),
            "plain_per_message_ms": round(pwall / 2 * 1e3, 3),
            "batched_vs_plain": round((total * reps / wall) / (total * 2 / pwall), 3)}


def bench_sector_batch(torch, A, dev, stream, nmsg=65536, size=4096, reps=5):
    """Many independent equal messages, as a storage layer sees them: 65,536
    sectors of 4 KiB, each with its own AES-128 key and IV, one graph launch.
    CBC encryption is serial within a message, so the batch runs one
    message per lane; CBC decryption and XTS are block-parallel.  GB/s per
    mode, same bytes."""
    import numpy as np
    rng = np.random.default_rng(6)
    keys = np.zeros((2 * nmsg, 32), np.uint8)
    keys[:, :16] = rng.integers(0, 256, (2 * nmsg, 16), dtype=np.uint8)
    ivs = rng.integers(0, 256, (nmsg, 16), dtype=np.uint8)
    total = nmsg * size
    x = seedgen.data_torch(6, 0, total, dev)
    y = torch.empty(total + 16 * nmsg, dtype=torch.uint8, device=dev)   # GCM tags after the data
    res = {"workload": "%d messages of %d B, per-message AES-128 key and IV (XTS: key pair, one %d-byte data "
                       "unit per message; GCM: 96-bit IV, no additional data, 16-byte tag)" % (nmsg, size, size),
           "bytes": total}
    xts = np.stack([A.xts_ctr0(m, nmsg + m, size) for m in range(nmsg)])
    for name, mode, dec, ctr0 in (("cbc_encrypt", "cbc", 0, ivs), ("cbc_decrypt", "cbc", 1, ivs),
                                  ("xts_encrypt", "xts", 0, xts)):
        descs = A.make_descs(np.full(nmsg, size), keybits=128, mode=mode, decrypt=dec, ctr0=ctr0)
        b = A.Batch(descs, keys, x, y)
        r = leg(torch, stream, lambda: b.launch_graph(stream), total, reps, 2)
        b.close()
        res[name + "_GB/s"] = r["GB/s"]
        res[name + "_launch_us"] = r["launch_us"]
    gcm = np.zeros(nmsg, A.GCM_DESC_DTYPE)
    gcm["tag_off"] = total + 16 * np.arange(nmsg)
    descs = A.make_descs(np.full(nmsg, size), keybits=128, mode="gcm", ctr0=ivs)
    b = A.Batch(descs, keys, x, y, gcm=gcm)
    r = leg(torch, stream, lambda: b.launch_graph(stream), total, reps, 2)
    b.close()
    res["gcm_encrypt_GB/s"] = r["GB/s"]
    res["gcm_encrypt_launch_us"] = r["launch_us"]
    del x, y
    torch.cuda.empty_cache()
    return res


def bench_gcm_large_batch(torch, A, dev, stream, nmsg=8, size=64 << 20, reps=10):
    """GCM over a batch of large messages: 8 x 64 MiB, each with its own
    AES-128 key and 96-bit IV, no additional data, 16-byte tags after the
    data, one graph launch.  Messages of 2 MiB and more are encrypted and
    hashed in one pass (the library's default); the same batch in two passes
    (counter mode, then a hash pass that reads the ciphertext again) beside
    it.  GB/s over the median launch."""
    import numpy as np
    rng = np.random.default_rng(7)
    keys = np.zeros((nmsg, 32), np.uint8)
    keys[:, :16] = rng.integers(0, 256, (nmsg, 16), dtype=np.uint8)
    ivs = np.zeros((nmsg, 16), np.uint8)
    ivs[:, :12] = rng.integers(0, 256, (nmsg, 12), dtype=np.uint8)
    total = nmsg * size
    x = seedgen.data_torch(7, 0, total, dev)
    y = torch.empty(total + 16 * nmsg, dtype=torch.uint8, device=dev)
    g = np.zeros(nmsg, A.GCM_DESC_DTYPE)
    g["tag_off"] = total + 16 * np.arange(nmsg)
    g["tag_bytes"] = 16
    descs = A.make_descs(np.full(nmsg, size), keybits=128, mode="gcm", ctr0=ivs)
    res = {"workload": "%d GCM messages of %d MiB, per-message AES-128 key and 96-bit IV, no additional data, "
                       "16-byte tags, encrypt" % (nmsg, size >> 20), "bytes": total}
    for name, two_pass in (("one_pass", False), ("two_pass", True)):
        b = A.Batch(descs, keys, x, y, gcm=g, gcm_two_pass=two_pass)
        r = leg(torch, stream, lambda: b.launch_graph(stream), total, reps, 2)
        b.close()
        res[name + "_GB/s"] = r["GB/s"]
        res[name + "_launch_us"] = r["launch_us"]
    del x, y
    torch.cuda.empty_cache()
    return res


def bench_served(torch, A, dev, plain_ctr_gbs, nreq, warm=1000,
                 loads=(0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2)):
    """The served workload: Poisson arrivals of CTR requests (70 % encrypt,
    30 % decrypt), sizes log-uniform in [64 B, 64 MiB], AES-128/256 half and
    half, each with its own key and nonce, admitted against an 8 GiB HBM
    budget on 4 streams.  The loop's capacity is measured first: the same
    requests all waiting at once, completed bytes over the span (payload
    fill included).  The arrival rate is then swept over offered loads
    rho = rate x mean size / capacity.  Latency runs from arrival to
    completion seen by the loop; the first `warm` requests of each run are
    excluded.  Each point also reports the payload fill's share of the
    launches' device time (HIP events around the fill and the batch)."""
    import numpy as np
    lo, hi = 64, 1 << 26
    mean = (hi - lo) / np.log(hi / lo)
    f, keys = seedgen.served_requests(5, nreq + warm, rate=1.0, lo=lo, hi=hi)
    base = np.zeros(nreq + warm, A.REQUEST_DTYPE)
    for k, v in f.items():
        base[k] = v
    cfg = A.serve_cfg(streams=4, budget_bytes=8 << 30, max_batch_msgs=4096)
    srv = A.Server(keys, cfg, device=dev)

    def fill_share(st):
        tot = st["fill_device_s"] + st["cipher_device_s"]
        return round(st["fill_device_s"] / tot, 4) if tot > 0 else None

    # capacity: everything waiting from the start (warm-up run first)
    r = base.copy()
    r["arrival_s"] = 0.0
    srv.run(r)
    res, st = srv.run(r)
    capacity_gbs = float(r["nbytes"].sum()) / float(res["latency_s"].max()) / 1e9
    capacity = {"GB/s": round(capacity_gbs, 1), "launches": st["launches"],
                "fill_share_of_device_time": fill_share(st),
                "plain_ctr_GB/s": round(plain_ctr_gbs, 1) if plain_ctr_gbs else None,
                "note": "all requests waiting at once: completed payload bytes over the span, payload fill "
                        "included; plain_ctr is the single-buffer CTR rate for the same 128/256 mix"}
    points = []
    for rho in loads:
        rate = rho * capacity_gbs * 1e9 / mean
        r = base.copy()
        r["arrival_s"] = base["arrival_s"] / rate
        res, st = srv.run(r)
        m = res[warm:]
        rm = r[warm:]
        t_first = float(rm["arrival_s"][0])
        t_last = float((rm["arrival_s"] + m["latency_s"]).max())
        points.append({"offered_load": rho, "arrival_rate_per_s": round(rate, 1),
                       "offered_GB/s": round(rho * capacity_gbs, 1),
                       "completed_GB/s": round(float(rm["nbytes"].sum()) / (t_last - t_first) / 1e9, 1),
                       "p50_ms": round(float(np.percentile(m["latency_s"], 50)) * 1e3, 3),
                       "p99_ms": round(float(np.percentile(m["latency_s"], 99)) * 1e3, 3),
                       "p50_admit_wait_ms": round(float(np.percentile(m["admit_s"], 50)) * 1e3, 3),
                       "launches": st["launches"], "max_inflight_reqs": st["max_inflight_reqs"],
                       "fill_share_of_device_time": fill_share(st)})
    # the same requests in GCM (no additional data; tags after the data):
    # the loop's GCM capacity measured the same way, then arrivals at half of
    # it and at half the CTR capacity
    rg = base.copy()
    rg["mode"] = A.AES_MODE_GCM
    rg["arrival_s"] = 0.0
    res, st = srv.run(rg)
    gcm_capacity_gbs = float(rg["nbytes"].sum()) / float(res["latency_s"].max()) / 1e9

    def gcm_point(rate, label, rho):
        r = base.copy()
        r["mode"] = A.AES_MODE_GCM
        r["arrival_s"] = base["arrival_s"] / rate
        res, st = srv.run(r)
        m, rm = res[warm:], r[warm:]
        t_first = float(rm["arrival_s"][0])
        t_last = float((rm["arrival_s"] + m["latency_s"]).max())
        return {label: rho, "arrival_rate_per_s": round(rate, 1),
                "completed_GB/s": round(float(rm["nbytes"].sum()) / (t_last - t_first) / 1e9, 1),
                "p50_ms": round(float(np.percentile(m["latency_s"], 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(m["latency_s"], 99)) * 1e3, 3),
                "launches": st["launches"],
                "encryptions_tagged": int((res["authentic"][r["decrypt"] == 0] == 1).sum()),
                "decryptions_rejected": int((res["authentic"][r["decrypt"] == 1] == 0).sum())}

    gcm = {"mode": "GCM", "capacity_GB/s": round(gcm_capacity_gbs, 1),
           "points": [gcm_point(0.5 * gcm_capacity_gbs * 1e9 / mean, "offered_load_of_gcm_capacity", 0.5),
                      gcm_point(0.5 * capacity_gbs * 1e9 / mean, "offered_load_of_ctr_capacity", 0.5)],
           "note": "capacity: all requests waiting at once, as for CTR; decryptions of the random payloads "
                   "must all fail authentication"}
    # the loop's own ceiling: every request 64 bytes and already waiting, so
    # admission, planning and completion are all there is to do
    r = base.copy()
    r["arrival_s"] = 0.0
    r["nbytes"] = 64
    res, st = srv.run(r)
    span = float(res["latency_s"].max())
    loop_rate = {"requests": len(r), "request_bytes": 64, "req_per_s": round(len(r) / span, 1),
                 "launches": st["launches"], "not_ok": int((res["status"] != 0).sum())}
    del srv
    torch.cuda.empty_cache()
    return {"workload": "Poisson CTR requests, 70/30 encrypt/decrypt, log-uniform 64 B..64 MiB, "
                        "AES-128/256 50/50, per-request key and nonce, 8 GiB HBM budget, 4 streams",
            "requests_per_point": nreq, "warmup_requests": warm, "tile_blocks": cfg.tile_blocks,
            "capacity_GB/s": round(capacity_gbs, 1), "capacity": capacity, "points": points,
            "gcm": gcm, "max_admitted": loop_rate}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(each GPU would encrypt its own shard with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1403_7295_amd import aesgpu as A

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.nbytes
    key128 = seedgen.key(2, 0, 128)
    ctr0 = seedgen.nonce(2, 0)
    x = seedgen.data_torch(2, 0, n, dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)

    def step():
        rk, nr = A.aes_expand_key(key128)
        A.aes_encrypt(x, y, n, rk, nr, A.AES_MODE_ECB, stream=stream)

    kstats = {}
    wall, kern = timed_launches(torch, stream, step, args.steps, args.warmup, stats=kstats)
    launch = A.aes_get_launch(n, A.AES_MODE_ECB, False, 10)
    value = n * args.steps / wall / 1e9
    nblocks = n // 16

    hbm_achieved = 2 * n / kern / 1e9
    lk = lookups_per_block(10) * nblocks
    issue_achieved = lk / kern / 1e12
    traffic = measured_traffic(launch)
    roof_hbm = {"bound": "hbm", "achieved": round(hbm_achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic}
    roof_issue = {"bound": "alu", "achieved": round(issue_achieved, 3),
                  "peak": round(LDS_PEAK_TLOOKUPS, 3), "unit": "Tlookup/s",
                  "frac": round(issue_achieved / LDS_PEAK_TLOOKUPS, 4), "traffic": traffic,
                  "note": "LDS table lookups (16 per round per block); peak = 256 CUs x 2.4 GHz "
                          "x 32 lanes per clock"}
    binding = roof_issue if roof_issue["frac"] >= roof_hbm["frac"] else roof_hbm

    out = {
        "metric": "AES-128 ECB encrypt GB/s @1 GiB",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (SplitMix64-seeded uniform random bytes, generated on the device)",
        "config": {"workload": "AES-128 ECB encrypt of a 1 GiB device-resident buffer, one seeded key",
                   "nbytes": n, "blocks": nblocks, "key_bits": 128, "mode": "ECB",
                   "launch": launch},
        "gbps": round(8 * value, 1),
        "kernel_ms": round(kern * 1e3, 4),
        "kernel_us": kstats,
        "roofline": binding,
        "roofline_hbm": roof_hbm,
        "roofline_issue": roof_issue,
    }

    if not args.no_secondary:
        sec = {}
        key256 = seedgen.key(2, 0, 256)
        for name, key, mode, dec in (("aes128_ctr_enc", key128, A.AES_MODE_CTR, False),
                                     ("aes128_ecb_dec", key128, A.AES_MODE_ECB, True),
                                     ("aes128_ctr_dec", key128, A.AES_MODE_CTR, True),
                                     ("aes128_cbc_dec", key128, A.AES_MODE_CBC, True),
                                     ("aes256_ecb_enc", key256, A.AES_MODE_ECB, False),
                                     ("aes256_ctr_enc", key256, A.AES_MODE_CTR, False)):
            rk, nr = A.aes_expand_key(key)
            fn = A.aes_decrypt if dec else A.aes_encrypt
            sec[name] = leg(torch, stream, lambda: fn(x, y, n, rk, nr, mode, ctr0=ctr0, stream=stream), n)
        rk, nr = A.aes_expand_key(key128)
        A.aes_set_launch(layout=2)
        try:
            for name, mode in (("aes128_ecb_enc_bitsliced", A.AES_MODE_ECB),
                               ("aes128_ctr_enc_bitsliced", A.AES_MODE_CTR)):
                sec[name] = leg(torch, stream,
                                lambda: A.aes_encrypt(x, y, n, rk, nr, mode, ctr0=ctr0, stream=stream), n)
        finally:
            A.aes_set_launch(None)
        # XTS over 512-byte and 4 KiB data units (tweak key: the next seeded key)
        for bits, key in ((128, key128), (256, key256)):
            rk1, nr = A.aes_expand_key(key)
            rk2, _ = A.aes_expand_key(seedgen.key(2, 1, bits))
            for unit in (512, 4096):
                for dec in (False, True):
                    fn = A.aes_xts_decrypt if dec else A.aes_xts_encrypt
                    sec["xts%d_%s_unit%d" % (bits, "dec" if dec else "enc", unit)] = leg(
                        torch, stream, lambda: fn(x, y, n, rk1, rk2, nr, unit, 0, stream=stream), n)
        # GCM (CTR with the GHASH tag fused), 16 bytes of additional data
        gws = torch.empty(A.aes_gcm_workspace_size(), dtype=torch.uint8, device=dev)
        gtag = torch.empty(16, dtype=torch.uint8, device=dev)
        gok = torch.empty(1, dtype=torch.int32, device=dev)
        gaad = torch.zeros(16, dtype=torch.uint8, device=dev)
        giv = seedgen.nonce(2, 3)[:12]   # the standard 96-bit IV
        for bits, key in ((128, key128), (256, key256)):
            rk, nr = A.aes_expand_key(key)
            sec["aes%d_gcm_enc" % bits] = leg(torch, stream, lambda: A.aes_gcm_encrypt(
                x, y, n, gaad, 16, rk, nr, giv, gtag, gws, stream=stream), n)
            sec["aes%d_gcm_dec" % bits] = leg(torch, stream, lambda: A.aes_gcm_decrypt(
                y, x, n, gaad, 16, rk, nr, giv, gtag, 16, gok, gws, stream=stream), n)
        # GMAC: the tag of 1 GiB of additional data with no plaintext
        rk, nr = A.aes_expand_key(key128)
        sec["aes128_gmac"] = leg(torch, stream, lambda: A.aes_gcm_encrypt(
            x, y, 0, x, n, rk, nr, giv, gtag, gws, stream=stream), n)
        # the decryptions above wrote the plaintext back into x
        # the 1 MiB case (AES-128 ECB): it stays in the caches between launches
        rk, nr = A.aes_expand_key(key128)
        sec["aes128_ecb_enc_1MiB"] = dict(leg(torch, stream, lambda: A.aes_encrypt(
            x, y, 1 << 20, rk, nr, A.AES_MODE_ECB, stream=stream), 1 << 20, 200, 10), cache_resident=True)
        # one GPU's share of the 1 GiB job if it were split over eight GPUs
        rk, nr = A.aes_expand_key(key128)
        share = n // 8
        sec["aes128_ecb_enc_eighth_share"] = dict(leg(torch, stream, lambda: A.aes_encrypt(
            x, y, share, rk, nr, A.AES_MODE_ECB, stream=stream), share, 40, 5), bytes=share)
        cp = leg(torch, stream, lambda: A.aes_copy(x, y, n, stream=stream), 2 * n)
        sec["copy_kernel"] = {"GB/s (read+write)": cp["GB/s"], "launch_us": cp["launch_us"]}
        sec["statistic"] = "GB/s over the median launch (HIP events); launch_us: every launch statistic"
        out["secondary"] = sec
        # the HBM fraction also against what a plain copy achieves on this device
        copy_gbs = cp["GB/s"]
        out["roofline_hbm"]["copy_GB/s"] = round(copy_gbs, 1)
        out["roofline_hbm"]["frac_of_copy"] = round(out["roofline_hbm"]["achieved"] / copy_gbs, 4)

    if not args.no_sweep:
        out["size_sweep"] = bench_size_sweep(torch, A, dev, stream)

    if not args.no_batched:
        out["batched"] = bench_batched(torch, A, dev, stream)
        out["sector_batch"] = bench_sector_batch(torch, A, dev, stream)
        out["gcm_large_batch"] = bench_gcm_large_batch(torch, A, dev, stream)

    if not args.no_served:
        plain = None
        if "secondary" in out:
            a, b = out["secondary"]["aes128_ctr_enc"]["GB/s"], out["secondary"]["aes256_ctr_enc"]["GB/s"]
            plain = 2.0 / (1.0 / a + 1.0 / b)     # half the bytes at each key size
        out["served"] = bench_served(torch, A, dev, plain, args.served_requests)

    # every table layout on the headline workload, each at its best blocks per
    # thread and workgroup size of the 1 GiB sweep (four tables x 32 copies,
    # two x 64, one x 64 with two workgroups per compute unit, four x 1)
    if not args.no_secondary:
        rk, nr = A.aes_expand_key(key128)
        lay = {}
        for layout, bpt in ((0, 4), (1, 4), (3, 2), (4, 4)):
            A.aes_set_launch(layout=layout, blocks_per_thread=bpt, wg_size=1024)
            try:
                cfg = A.aes_get_launch(n, A.AES_MODE_ECB, False, nr)
                lay["layout%d" % layout] = dict(leg(torch, stream, lambda: A.aes_encrypt(
                    x, y, n, rk, nr, A.AES_MODE_ECB, stream=stream), n), launch=cfg)
            finally:
                A.aes_set_launch(None)
        out["layouts"] = lay

    # the lookup rate the LDS accepts on this device, measured last: the
    # calibration kernel runs at a high clock and power, and measurements
    # taken right after it came out slowed
    lds = bench_lds_gather(torch, A, dev, stream)
    out["lds_gather"] = lds
    out["lds_gather_one_table"] = bench_lds_gather(torch, A, dev, stream, layout=3)
    roof_issue["measured_peak"] = lds["Tlookup/s"]
    roof_issue["frac_of_measured"] = round(issue_achieved / lds["Tlookup/s"], 4)
    roof_issue["measured_peak_note"] = ("the LDS calibration kernel in the same run: the cipher's lookup "
                                        "instructions without global memory, round keys or round-to-round "
                                        "dependence")

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_mib << 20)
        out["cpu_context"] = cpu_context_openssl()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
