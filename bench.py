#!/usr/bin/env python3
"""Benchmark of the suffix-array matching path on one MI355X.

One step = the whole device path over one batch already resident in HBM:
pack the ASCII reads to 2-bit words (sort them by prefix when the launch
settings say so), run the search kernel (prefix-table bracket or LDS tile,
LB search, RB search or longest-matched-prefix searches), store the 16-byte
results in input order.

Default workload (c4, the largest single-GPU one): a 250 Mbp order-3 Markov
reference with 10 % interspersed repeats (copies of twenty 300 bp elements
at 10 % divergence), and 64,000,000 reads of 150 bp (80 % sampled from the
reference at 1 % substitutions, 20 % random), all synthetic and seeded.

The timed steps write into a result buffer filled with a sentinel first, and
their output is compared with the instrumented run's and with the oracle's
on the CPU sample, so a timed kernel that skipped work would fail the run.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "paper": "10 Mbp order-3 Markov reference (GC 0.41) + 5% tandem repeats; 2,097,152 queries x 1024 bp "
             "(50% sampled at 0-1% substitutions, 50% random)",
    "c1": "1 Mbp i.i.d. reference; 100,000 reads x 25 bp (50% copied, a quarter of those with 1-2 substitutions, "
          "50% random)",
    "c2": "16 Mbp order-3 Markov reference (GC 0.41) + 5% tandem repeats; 4,000,000 reads x 100 bp "
          "(70% sampled at 0-2% substitutions, 30% random)",
    "c3": "16 Mbp order-3 Markov reference (GC 0.41) + 5% tandem repeats; 4,000,000 reads x U{20..300} bp "
          "(70% sampled at 0-2% substitutions, 30% random)",
    "c4": "250 Mbp order-3 Markov reference + 10% interspersed repeats (copies of 20 elements of 300 bp at 10% "
          "divergence); 64,000,000 reads x 150 bp (80% sampled at 1% substitutions, 20% random)",
}
CPU_SAMPLE_READS = 4_000_000
METRIC = "reads/s and matched Mbases/s at 1 GPU; p50/p99 request latency; HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "radix_sort.h"):
        h.update(open(os.path.join(ROOT, "paper_1303_3692_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--no-tune", action="store_true", help="use the built-in launch defaults")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel comparison")
    ap.add_argument("--no-e2e", action="store_true", help="skip the end-to-end timing from host memory")
    ap.add_argument("--serve-streams", type=int, default=2, help="--serve: pipelines the server runs at once")
    ap.add_argument("--serve-levels", default="0.5,0.8,0.95", help="--serve: loads relative to the offline rate")
    ap.add_argument("--no-graph", action="store_true", help="launch the kernels directly instead of replaying a graph")
    ap.add_argument("--prefix-bases", type=int, default=-1,
                    help="rebuild the index's prefix table for this many bases (0: none; default: the library's)")
    ap.add_argument("--per-length", action="store_true",
                    help="also time one batch call per distinct read length (default for c3)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before timing, copy this many MiB device to device once (a kernel of known traffic "
                         "for scaling memory counters)")
    ap.add_argument("--gen-workers", type=int, default=8,
                    help="processes that generate the reads (1: in this process, e.g. under a profiler)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1303_3692_amd", "tuning_cache.jsonl"),
                    help="autotuner cache (JSON lines); a hit skips the sweep")
    ap.add_argument("--paper", action="store_true",
                    help="paper-shape workload: 10 Mbp reference, 1024-base queries, sets of 512 to 2,097,152; "
                         "input / kernel / output / total per set (the columns of the paper's Table V)")
    ap.add_argument("--st", action="store_true",
                    help="suffix-tree comparison on the --config workload: the flattened suffix tree's search beside "
                         "the suffix-array path, results compared, index sizes")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark: open-loop Poisson requests over resident references")
    ap.add_argument("--serve-refs", default="c2,c4", help="references kept resident for --serve")
    ap.add_argument("--serve-linger-us", type=int, default=0,
                    help="--serve: a batch waits up to this long for max_batch_reads reads (0: starts at once)")
    ap.add_argument("--serve-batch-reads", type=int, default=1 << 20, help="--serve: reads per device batch")
    ap.add_argument("--serve-requests", type=int, default=4000, help="measured requests per load level")
    ap.add_argument("--serve-warmup", type=int, default=400, help="warm-up requests per load level")
    ap.add_argument("--serve-pool", type=int, default=800, help="distinct requests the streams draw from")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (reads shard across GPUs "
              "with no exchange step; this build runs and reports a single device)", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import gen

    if args.paper:
        args.config = "paper"
    if not args.serve:
        # inputs first: the generator forks workers, before this process uses the GPU
        t = time.perf_counter()
        ref = gen.make_reference(args.config)
        last = [time.perf_counter()]

        def progress(done, count):
            if time.perf_counter() - last[0] > 10 or done == count:
                last[0] = time.perf_counter()
                log(f"  reads generated: {done:,} of {count:,}")

        reads = gen.make_reads_parallel(ref, gen.READ_SPECS[args.config],
                                        workers=min(args.gen_workers, os.cpu_count() or 1), progress=progress)
        text = ref.ascii()
        log(f"workload {args.config}: n={ref.n} reads={reads.count} ({time.perf_counter() - t:.1f}s)")

    import torch

    import paper_1303_3692_amd as S

    if not os.path.exists(S.LIB_PATH):
        from paper_1303_3692_amd import build as B
        B.build()
    dev = torch.device("cuda:0")
    torch.cuda.init()
    if args.serve:
        return serve_bench(args, np, torch, gen, S)
    if args.paper:
        return paper_bench(args, np, torch, gen, S, ref, reads, text)
    if args.st:
        return st_bench(args, np, torch, gen, S, ref, reads, text)

    t = time.perf_counter()
    d = S.sa_build_device(text, 0)
    t_index = time.perf_counter() - t
    built = d.build_info()
    log(f"index: built on the device in {t_index:.2f}s ({built})")
    if args.prefix_bases >= 0:
        d.set_prefix_table(args.prefix_bases)
    index_bytes = d.index_bytes()
    log(f"index bytes: {index_bytes}")

    N = reads.count
    d_reads = torch.from_numpy(reads.data).to(dev)
    d_offs = torch.from_numpy(reads.offs).to(dev)
    d_out = torch.zeros((N, 4), dtype=torch.int32, device=dev)
    # a stream of our own: the default stream cannot be captured into a graph
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del src, dst

    tuned_ms = None
    if not args.no_tune:
        t = time.perf_counter()
        _, tuned_ms = S.sa_tune(d, d_reads, d_offs, stream=stream, cache_path=args.tune_cache)
        log(f"tuner: {time.perf_counter() - t:.1f}s -> {S.cfg(d).as_dict()} ({tuned_ms:.3f} ms)")
    cfg = S.cfg(d)
    cfg.use_graph = 0 if args.no_graph else 1

    def run_steps(c, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            S.match_batch_dev(d, d_reads, d_offs, d_out, stream=stream, config=c)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def stage_times(c, k):
        cp = S.cfg(d, **c.as_dict())
        cp.profile = 1
        acc = {"pack": 0.0, "sort": 0.0, "search": 0.0, "total": 0.0}
        for _ in range(k):
            S.match_batch_dev(d, d_reads, d_offs, d_out, stream=stream, config=cp)
            st = S.sa_stage_times(d, stream)
            for key in acc:
                acc[key] += st[key] / k
        return acc

    def counts(c):
        cc = S.cfg(d, **c.as_dict())
        cc.count = 1
        S.match_batch_dev(d, d_reads, d_offs, d_out, stream=stream, config=cc)
        return S.sa_probe_counts(d, stream)

    lens = reads.lengths()

    def packs_inline(c):
        # the search kernel packs the reads itself (no pack pass) when the
        # batch is in input order and its tile plus one packing area per
        # wave fit in LDS (160 KB less room for static variables); an area
        # holds 64 slots of 2 * max_words + 1 16-byte pieces (codes and
        # flags) and a queue of 128 set-aside read ids (kernels.h)
        tile = ((1 << c.tile_levels) - 1) * 12
        area = (((64 * (2 * c.max_words + 1) + 4) * 6 + 8) + 15) // 16 * 16 + 4 * 128
        return (c.kernel == S.SA_KERNEL_TUNED and c.inline_pack == 1 and c.sort == 0 and
                ((tile + 15) // 16 * 16 + (c.block // 64) * area) <= 160 * 1024 - 256)

    packed_bytes = int(((lens + 3) // 4).sum())
    ascii_bytes = int(lens.sum()) + 8 * N

    def probe_bytes(cnt):
        # per global probe a 4-byte SA entry plus the 8-byte words it
        # compares (row-record words and text words); per prefix-table
        # lookup its 16-byte entry
        return 4 * cnt["global_probes"] + 8 * (cnt["text_words"] + cnt["key_words"]) + 16 * cnt["table_lookups"]

    def alg_bytes(cnt, c, ingest=False):
        # per read: the 2-bit packed read (ceil(m/4) bytes) + the 16-byte
        # result + its probes.  ingest=True counts instead what the fused
        # kernel reads as input: the ASCII bytes and an 8-byte offset
        read_bytes = ascii_bytes if (ingest and packs_inline(c)) else packed_bytes
        return read_bytes + 16 * N + probe_bytes(cnt)

    SENTINEL = -7

    def timed_output(c, k):
        # fill the results with a sentinel outside the timed region, run k
        # steps, and return the elapsed time and what the timed steps wrote
        d_out.fill_(SENTINEL)
        el = run_steps(c, k)
        res = d_out.cpu().numpy()
        assert (res[:, 0] != SENTINEL).all() and (res[:, 3] != SENTINEL).all(), "timed steps left results unwritten"
        return el, res

    # ---- tuned path
    cnt = counts(cfg)
    check = d_out.cpu().numpy()
    run_steps(cfg, args.warmup)
    elapsed, out = timed_output(cfg, args.steps)
    ms_step = 1000.0 * elapsed / args.steps
    assert (out == check).all(), "instrumented and timed runs disagree"
    stages = stage_times(cfg, max(3, min(args.steps, 10)))
    matched = int(out[:, 2].astype(np.int64).sum())
    exact = float((out[:, 3] & 1).mean())
    log(f"tuned: {ms_step:.3f} ms/step, stages {stages}")

    # ---- plain kernel side by side
    plain = None
    if not args.no_plain:
        pc = S.cfg(d, kernel=S.SA_KERNEL_PLAIN)
        pcnt = counts(pc)
        run_steps(pc, 1)
        pk = max(2, args.steps // 4)
        pel, pout = timed_output(pc, pk)
        assert (pout[:, :3] == out[:, :3]).all() and ((pout[:, 3] & 1) == (out[:, 3] & 1)).all(), \
            "plain and tuned kernels disagree"
        pst = stage_times(pc, 3)
        plain = {"reads_per_s": N * pk / pel, "ms_per_step": 1000.0 * pel / pk, "search_ms": pst["search"],
                 "global_probes_per_read": pcnt["global_probes"] / N,
                 "alg_bytes_per_read": alg_bytes(pcnt, pc) / N,
                 "search_GBps_alg": alg_bytes(pcnt, pc) / (pst["search"] * 1e-3) / 1e9}
        log(f"plain: {plain}")

    # ---- one call per distinct read length (the unbatched form)
    per_length = None
    if args.per_length or args.config == "c3":
        groups = []
        for L in np.unique(lens):
            idx = np.nonzero(lens == L)[0]
            starts = reads.offs[idx]
            data_l = (reads.data[starts[:, None] + np.arange(L)[None, :]].reshape(-1) if L > 0
                      else np.zeros(1, np.uint8))
            offs_l = np.arange(len(idx) + 1, dtype=np.int64) * int(L)
            groups.append((torch.from_numpy(np.ascontiguousarray(data_l)).to(dev), torch.from_numpy(offs_l).to(dev),
                           torch.zeros((len(idx), 4), dtype=torch.int32, device=dev)))
        lc = S.cfg(d, **cfg.as_dict())
        lc.nbuckets = 1
        lc.bucket_edge[0] = S.SA_MAX_READ
        lc.use_graph = 0

        def per_length_steps(k):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                for g_reads, g_offs, g_out in groups:
                    S.match_batch_dev(d, g_reads, g_offs, g_out, stream=stream, config=lc)
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        per_length_steps(1)
        pk = max(2, args.steps // 4)
        pel = per_length_steps(pk)
        per_length = {"calls_per_step": len(groups), "ms_per_step": round(1000.0 * pel / pk, 3),
                      "reads_per_s": round(N * pk / pel, 1)}
        log(f"per-length: {per_length}")
        del groups
        # each 32-base length class as a batch of its own, in the batched
        # configuration: what every class costs, against the whole batch
        words = np.maximum(1, (lens + 31) // 32)
        per_class = []
        for w in np.unique(words):
            idx = np.nonzero(words == w)[0]
            ln = lens[idx]
            offs_w = np.zeros(len(idx) + 1, dtype=np.int64)
            np.cumsum(ln, out=offs_w[1:])
            src = np.repeat(reads.offs[idx] - offs_w[:-1], ln) + np.arange(int(offs_w[-1]), dtype=np.int64)
            cr = torch.from_numpy(np.ascontiguousarray(reads.data[src])).to(dev)
            co = torch.from_numpy(offs_w).to(dev)
            cout = torch.zeros((len(idx), 4), dtype=torch.int32, device=dev)
            S.match_batch_dev(d, cr, co, cout, stream=stream, config=lc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(pk):
                S.match_batch_dev(d, cr, co, cout, stream=stream, config=lc)
            torch.cuda.synchronize()
            ms_c = 1000.0 * (time.perf_counter() - t0) / pk
            per_class.append({"bases": f"{32 * int(w) - 31}-{32 * int(w)}", "reads": int(len(idx)),
                              "ms": round(ms_c, 4), "reads_per_s": round(len(idx) / (ms_c * 1e-3), 1)})
            del cr, co, cout
        per_length["per_class"] = per_class
        per_length["per_class_ms_total"] = round(sum(c["ms"] for c in per_class), 3)
        log(f"per length class: {per_class}")

    # ---- locate (positions of exact reads, at most 16 per read) on this step's hits
    loc_offs = torch.zeros(N + 1, dtype=torch.int64, device=dev)
    try:
        S.locate_dev(d, d_out, 16, 0, loc_offs, torch.zeros(1, dtype=torch.int32, device=dev), stream=stream)
    except S.SaError as err:
        if err.code != S.SA_ENOSPC:
            raise
    total = int(loc_offs[-1].item())
    loc_pos = torch.zeros(max(1, total), dtype=torch.int32, device=dev)
    S.locate_dev(d, d_out, 16, 0, loc_offs, loc_pos, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        S.locate_dev(d, d_out, 16, 0, loc_offs, loc_pos, stream=stream)
    torch.cuda.synchronize()
    loc_ms = (time.perf_counter() - t) / 5 * 1000
    locate = {"cap": 16, "positions": total, "ms": round(loc_ms, 4),
              "positions_per_s": round(total / (loc_ms * 1e-3), 1)}
    log(f"locate: {locate}")
    del loc_offs, loc_pos

    B = alg_bytes(cnt, cfg)
    B_ingest = alg_bytes(cnt, cfg, ingest=True)
    achieved = B / (stages["search"] * 1e-3) / 1e9
    # HBM traffic per launch and the L2 hit rate from the committed
    # rocprofv3 counters, only when they were taken on these kernel sources
    # and this workload
    traffic, l2_hit = None, None
    counters = os.path.join(ROOT, "profiles", f"search_tuned_{args.config}_counters.json")
    if os.path.exists(counters):
        prof = json.load(open(counters))
        if prof.get("kernel_src") == kernel_source_hash() and prof.get("workload") == args.config:
            traffic = round(prof["traffic_bytes"])
            l2_hit = prof.get("l2_hit_rate")
    touched = cnt["touched_bytes"]
    # the search's scattered accesses (64-byte segments of the index its
    # loads address) against the rate this device serves random 16-byte
    # loads from a table the size of the row records
    scattered = cnt["index_segments"]
    ceiling = S.sa_random_read_rate(0, max(8, min(28, int(np.ceil(np.log2(max(2, len(d))))))))
    scattered_rate = scattered / (stages["search"] * 1e-3)
    log(f"random 16-byte loads: {ceiling / 1e9:.1f} G/s; search scattered segments {scattered_rate / 1e9:.1f} G/s")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "l2_hit_rate": l2_hit,
                "kernel": "search_tuned_kernel", "packs_reads": packs_inline(cfg),
                "alg_bytes_per_launch": B, "alg_bytes_per_read": round(B / N, 2),
                # the same with the input counted as the fused kernel reads it (ASCII + offsets)
                "ingest_alg_bytes_per_launch": B_ingest,
                "frac_ingest_inclusive": round(B_ingest / (stages["search"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                "launch_ms": round(stages["search"], 4), "kernel_src": kernel_source_hash(),
                # bytes touched: 64-byte segments addressed per wave access, counted by the instrumented kernel
                "touched_bytes_per_launch": touched, "touched_GBps": round(touched / (stages["search"] * 1e-3) / 1e9, 2),
                "touched_frac": round(touched / (stages["search"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                # measured random-access ceiling (G 16-byte loads/s) and the
                # search's scattered 64-byte segments per second against it
                "random_ceiling_G_per_s": round(ceiling / 1e9, 2),
                "scattered_G_per_s": round(scattered_rate / 1e9, 2),
                "random_frac": round(scattered_rate / ceiling, 4)}

    # ---- end to end from host memory (match_batch: reads copied in, results
    # copied out, over PCIe; not the headline, which starts from HBM)
    e2e = None
    if not args.no_e2e:
        S.match_batch(d, reads.data, reads.offs)
        t = time.perf_counter()
        for _ in range(3):
            S.match_batch(d, reads.data, reads.offs)
        t_e2e = (time.perf_counter() - t) / 3
        e2e = {"ms_per_batch": round(1000 * t_e2e, 3), "reads_per_s": round(N / t_e2e, 1),
               "input_bytes": int(len(reads.data) + 8 * (N + 1)), "output_bytes": 16 * N}
        log(f"end to end from host memory: {e2e}")

    # ---- CPU baseline: the oracle's search phase on the host cores, on a
    # bounded sample of the batch (its first reads)
    cpu = None
    if not args.no_cpu:
        from oracle import oracle
        t = time.perf_counter()
        osa = S.sa_download(d).suffix_array()
        ok = oracle.sa_check(text, osa) == 0  # a permutation with sorted neighbours is the suffix array
        t_chk = time.perf_counter() - t
        assert ok, "device suffix array failed the oracle's check"
        ns = min(N, CPU_SAMPLE_READS)
        threads = oracle.max_threads()
        t = time.perf_counter()
        want = oracle.match(text, osa, reads.data[:reads.offs[ns]], reads.offs[:ns + 1], nthreads=threads)
        t_match = time.perf_counter() - t
        got = out[:ns]
        same = bool((want[:, :3] == got[:, :3]).all() and (want[:, 3] == (got[:, 3] & 1)).all())
        # and on one core, over a smaller sample
        n1 = min(ns, CPU_SAMPLE_READS // 16)
        t = time.perf_counter()
        want1 = oracle.match(text, osa, reads.data[:reads.offs[n1]], reads.offs[:n1 + 1], nthreads=1)
        t_one = time.perf_counter() - t
        same = same and bool((want1 == want[:n1]).all())
        cpu = {"value": round(ns / t_match, 1), "unit": "reads/s", "cores": threads, "kind": "oracle",
               "sample": f"the first {ns:,} of {N:,} reads; oracle search phase only, over the device-built suffix "
                         f"array after the oracle checked it sorted ({t_chk:.1f}s, untimed)",
               "matches_gpu": same,
               "one_core": {"value": round(n1 / t_one, 1), "unit": "reads/s", "sample": f"the first {n1:,} reads"}}
        log(f"cpu oracle: {cpu}")

    value = N * args.steps / elapsed
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "reads/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic (seeded generators, no external data)",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "reference_bp": ref.n, "reads": N,
                   "global_batch": N, "parallelism": "single GPU", "launch": cfg.as_dict()},
        "matched_mbases_per_s": round(matched * args.steps / elapsed / 1e6, 2),
        "query_mbases_per_s": round(int(lens.sum()) * args.steps / elapsed / 1e6, 2),
        "exact_fraction": round(exact, 5),
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "probes_per_read": {"global": round(cnt["global_probes"] / N, 3), "lds": round(cnt["tile_probes"] / N, 3),
                            "text_words": round(cnt["text_words"] / N, 3), "key_words": round(cnt["key_words"] / N, 3),
                            "table_lookups": round(cnt["table_lookups"] / N, 3),
                            "touched_bytes": round(cnt["touched_bytes"] / N, 1),
                            # memory requests of the searches: 64-byte segments of the index that the
                            # wave's loads address (scattered), and index loads issued per lane
                            "index_segments": round(cnt["index_segments"] / N, 3),
                            "index_loads": round(cnt["index_loads"] / N, 3)},
        "index": {"device_build_s": round(t_index, 3), "sort_rounds": built["steps"],
                  "sorted_pairs": built["sorted_pairs"],
                  # device bytes the timed (tuned) path reads, by part; the plain kernel reads text + suffix array
                  "bytes": index_bytes, "tuned_path_bytes": sum(index_bytes.values()),
                  "plain_path_bytes": index_bytes["text"] + index_bytes["suffix_array"]},
        "plain": plain,
        "speedup_vs_plain": round(value / plain["reads_per_s"], 3) if plain else None,
        "per_length": per_length,
        "speedup_vs_per_length": round(value / per_length["reads_per_s"], 3) if per_length else None,
        "locate": locate,
        "end_to_end_from_host": e2e,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q * (len(xs) - 1)))))
    return xs[k]


def paper_bench(args, np, torch, gen, S, ref, reads, text):
    """The paper's experiment shape (Section V, Table V): one 10^7-base
    reference, query sets of 512 .. 2,097,152 reads of 1024 bases.  Per set:
    input (host-to-device copy of the reads from pinned memory), kernel (the
    whole device pipeline), output (device-to-host copy of the 16-byte
    results) and total, each the median of 5 runs timed with HIP events on
    one stream.  The index is resident (built once, timed apart)."""
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    d = S.sa_build_device(text, 0)
    t_index = time.perf_counter() - t
    log(f"index built on the device in {t_index:.2f}s")
    N = reads.count
    h_reads = torch.from_numpy(reads.data).pin_memory()
    h_offs = torch.from_numpy(reads.offs).pin_memory()
    d_reads = torch.empty(len(reads.data), dtype=torch.uint8, device=dev)
    d_offs = torch.empty(N + 1, dtype=torch.int64, device=dev)
    d_out = torch.empty((N, 4), dtype=torch.int32, device=dev)
    h_out = torch.empty((N, 4), dtype=torch.int32).pin_memory()
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    d_reads.copy_(h_reads)
    d_offs.copy_(h_offs)
    t = time.perf_counter()
    _, tuned_ms = S.sa_tune(d, d_reads, d_offs, stream=stream, cache_path=args.tune_cache)
    log(f"tuner: {time.perf_counter() - t:.1f}s -> {S.cfg(d).as_dict()} ({tuned_ms:.3f} ms)")
    cfg = S.cfg(d)
    cfg.use_graph = 1  # one captured launch sequence per set size
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    rows = []
    Q = 512
    while Q <= N:
        nb = int(reads.offs[Q])
        samples = []
        for rep in range(6):
            ev[0].record(stream)
            d_reads[:nb].copy_(h_reads[:nb], non_blocking=True)
            d_offs[:Q + 1].copy_(h_offs[:Q + 1], non_blocking=True)
            ev[1].record(stream)
            S.match_batch_dev(d, d_reads, d_offs[:Q + 1], d_out, nreads=Q, stream=stream, config=cfg)
            ev[2].record(stream)
            h_out[:Q].copy_(d_out[:Q], non_blocking=True)
            ev[3].record(stream)
            stream.synchronize()
            if rep:
                samples.append([ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3]),
                                ev[0].elapsed_time(ev[3])])
        med = [sorted(x[k] for x in samples)[len(samples) // 2] for k in range(4)]
        rows.append({"queries": Q, "input_ms": round(med[0], 4), "kernel_ms": round(med[1], 4),
                     "output_ms": round(med[2], 4), "total_ms": round(med[3], 4),
                     "kernel_queries_per_s": round(Q / (med[1] * 1e-3), 1),
                     "total_queries_per_s": round(Q / (med[3] * 1e-3), 1)})
        log(f"Q={Q}: {rows[-1]}")
        Q *= 2
    out = h_out.numpy()
    # parity on a sample, the oracle searching the device array after checking it
    from oracle import oracle
    osa = S.sa_download(d).suffix_array()
    assert oracle.sa_check(text, osa) == 0, "device suffix array failed the oracle's check"
    ns = min(N, 65536)
    threads = oracle.max_threads()
    t = time.perf_counter()
    want = oracle.match(text, osa, reads.data[:reads.offs[ns]], reads.offs[:ns + 1], nthreads=threads)
    t_match = time.perf_counter() - t
    same = bool((want[:, :3] == out[:ns, :3]).all() and (want[:, 3] == (out[:ns, 3] & 1)).all())
    assert same, "device results differ from the oracle on the sample"
    cpu = {"value": round(ns / t_match, 1), "unit": "queries/s", "cores": threads, "kind": "oracle",
           "sample": f"the first {ns:,} of {N:,} queries; oracle search phase only", "matches_gpu": same}
    log(f"cpu oracle: {cpu}")
    last = rows[-1]
    line = {
        "metric": "queries/s, whole device pipeline, 1024-base queries (the paper's Table V shape)",
        "value": last["kernel_queries_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": 5, "warmup": 1,
        "ms_per_step": last["kernel_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic (seeded generators, no external data)",
        "config": {"workload": f"paper: {WORKLOADS['paper']}", "reference_bp": ref.n, "launch": cfg.as_dict()},
        "exact_fraction": round(float((out[:, 3] & 1).mean()), 5),
        "index": {"device_build_s": round(t_index, 3)},
        "sets": rows, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def st_bench(args, np, torch, gen, S, ref, reads, text):
    """The paper's comparison (Sections III and V): the same reads searched
    through a flattened suffix tree and through the suffix array, device
    time per batch with HIP events on one stream, results compared read by
    read, and the device bytes of each index as searched."""
    dev = torch.device("cuda:0")
    d = S.sa_build_device(text, 0)
    t = time.perf_counter()
    st = S.st_build(S.sa_download(d))
    t_st = time.perf_counter() - t
    sd = S.st_upload(st, d)
    log(f"suffix tree: {st.node_count()} nodes, built on the host in {t_st:.1f}s")
    N = reads.count
    d_reads = torch.from_numpy(reads.data).to(dev)
    d_offs = torch.from_numpy(reads.offs).to(dev)
    out_sa = torch.zeros((N, 4), dtype=torch.int32, device=dev)
    out_st = torch.zeros((N, 4), dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    S.sa_tune(d, d_reads, d_offs, stream=stream, cache_path=args.tune_cache)
    cfg = S.cfg(d)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, k):
        fn()
        ev[0].record(stream)
        for _ in range(k):
            fn()
        ev[1].record(stream)
        stream.synchronize()
        return ev[0].elapsed_time(ev[1]) / k

    ms_sa = timed(lambda: S.match_batch_dev(d, d_reads, d_offs, out_sa, stream=stream, config=cfg), args.steps)
    ms_st = timed(lambda: S.st_match_batch_dev(sd, d_reads, d_offs, out_st, stream=stream), args.steps)
    same = bool((out_sa.cpu().numpy() == out_st.cpu().numpy()).all())
    assert same, "suffix-tree and suffix-array results differ"
    out_pl = torch.zeros((N, 4), dtype=torch.int32, device=dev)
    pc = S.cfg(d, kernel=S.SA_KERNEL_PLAIN)
    ms_pl = timed(lambda: S.match_batch_dev(d, d_reads, d_offs, out_pl, stream=stream, config=pc), max(2, args.steps // 4))
    pl = out_pl.cpu().numpy()
    sa_out = out_sa.cpu().numpy()
    assert (pl[:, :3] == sa_out[:, :3]).all() and ((pl[:, 3] & 1) == (sa_out[:, 3] & 1)).all(), "plain kernel differs"
    # device bytes each path reads: the tuned path every part of the index,
    # the plain kernel (the paper's search) the text and the suffix array,
    # the tree its nodes, the suffix array (leaves) and the text
    ib = d.index_bytes()
    tuned_bytes = sum(ib.values())
    sa_bytes = ib["text"] + ib["suffix_array"]
    st_bytes = st.device_bytes()
    line = {
        "metric": "reads/s: flattened suffix tree vs suffix array, same reads, identical results",
        "value": round(N / (ms_st * 1e-3), 1), "unit": "reads/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(ms_st, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic (seeded generators, no external data)",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "reference_bp": ref.n},
        "suffix_tree": {"ms_per_batch": round(ms_st, 4), "reads_per_s": round(N / (ms_st * 1e-3), 1),
                        "nodes": st.node_count(), "device_bytes": st.device_bytes(),
                        "host_build_s": round(t_st, 2)},
        "suffix_array_tuned": {"ms_per_batch": round(ms_sa, 4), "reads_per_s": round(N / (ms_sa * 1e-3), 1),
                               "device_bytes": tuned_bytes, "bytes_by_part": ib, "launch": cfg.as_dict()},
        "suffix_array_plain": {"ms_per_batch": round(ms_pl, 4), "reads_per_s": round(N / (ms_pl * 1e-3), 1),
                               "device_bytes": sa_bytes},
        "plain_sa_bytes_over_st_bytes": round(sa_bytes / st_bytes, 4),
        "tuned_sa_bytes_over_st_bytes": round(tuned_bytes / st_bytes, 4),
        "identical": same,
    }
    print(json.dumps(line), flush=True)


def serve_bench(args, np, torch, gen, S):
    """Open-loop Poisson request streams over resident references, at three
    loads relative to the offline rate of the same request mix through the
    host entry point; latency runs from each request's scheduled arrival to
    its completion (steady clock on both sides)."""
    names = args.serve_refs.split(",")
    refs, dix = [], []
    for name in names:
        t = time.perf_counter()
        ref = gen.make_reference(name)
        d = S.sa_build_device(ref.ascii(), 0)
        refs.append(ref)
        dix.append(d)
        log(f"reference {name}: n={ref.n} ready in {time.perf_counter() - t:.1f}s")
    mixes = [gen.ReadSpec(60 + i, 0, 30, 300, 0.3, 0.0, 0.02) if name in ("c2", "c3") else
             gen.ReadSpec(60 + i, 0, 30, 300, 0.2, 0.01, 0.01) for i, name in enumerate(names)]

    # offline rate of the mix through match_batch (host buffers in, results out)
    total_reads, total_t = 0, 0.0
    for i, (ref, d) in enumerate(zip(refs, dix)):
        spec = gen.ReadSpec(mixes[i].cfg_id + 1000, 1 << 20, 30, 300, mixes[i].frac_random, mixes[i].rate_lo,
                            mixes[i].rate_hi)
        rd = gen.make_reads(ref, spec)
        # tune the index's launch settings on this mix (the server and the
        # host path both use the index's settings)
        dr = torch.from_numpy(rd.data).to("cuda:0")
        do = torch.from_numpy(rd.offs).to("cuda:0")
        S.sa_tune(d, dr, do, cache_path=args.tune_cache)
        del dr, do
        S.match_batch(d, rd.data, rd.offs)
        t = time.perf_counter()
        for _ in range(3):
            S.match_batch(d, rd.data, rd.offs)
        total_t += time.perf_counter() - t
        total_reads += 3 * rd.count
    x_off = total_reads / total_t
    mean_size = float(np.mean(gen.request_sizes(200_000, np.random.default_rng(7))))
    log(f"offline host-path rate on the mix: {x_off / 1e6:.1f} M reads/s; mean request {mean_size:.0f} reads")

    t = time.perf_counter()
    pool = gen.request_pool(refs, args.serve_pool)
    log(f"{len(pool)} distinct requests ({sum(r.count for _, r in pool)} reads) generated in "
        f"{time.perf_counter() - t:.1f}s")
    levels = []
    touched_per_read = None
    for k, rho in enumerate(float(x) for x in args.serve_levels.split(",")):
        lam = rho * x_off / mean_size
        nreq = args.serve_warmup + args.serve_requests
        stream = gen.request_stream(refs, nreq, lam, seed_sub=k, pool=pool)

        def serve(measure):
            # the client: native threads of the library submit each request
            # at its scheduled time (open loop), so no interpreter lock sits
            # in the measured loop; measure 1 times each batch's search
            # stage with events, measure 2 runs the instrumented kernels
            srv = S.Server(dix, max_batch_reads=args.serve_batch_reads, nstreams=args.serve_streams, measure=measure,
                           batch_linger_us=args.serve_linger_us)
            res = srv.replay([r.ref for r in stream], [r.reads.data for r in stream], [r.reads.offs for r in stream],
                             [int(r.t_arrival * 1e9) for r in stream], nthreads=32)
            tot = srv.stats()
            srv.destroy()
            return res, tot

        if touched_per_read is None:
            # bytes the served search kernels touch per read, from one
            # instrumented pass over this stream (its timing is not used)
            _, tot2 = serve(2)
            touched_per_read = tot2["touched_bytes"] / max(1, tot2["reads"])
            log(f"served search kernels: {touched_per_read:.1f} bytes touched per read")
        (outs, sched, stats), tot = serve(1)
        done = {i: (stats[i]["status"], stats[i]) for i in range(nreq)}
        meas = range(args.serve_warmup, nreq)
        lat = [(done[i][1]["t_done_ns"] - int(sched[i])) / 1e6 for i in meas if done[i][0] == S.SA_OK]
        reads_meas = sum(stream[i].reads.count for i in meas)
        span = (max(done[i][1]["t_done_ns"] for i in meas) - min(int(sched[i]) for i in meas)) / 1e9
        late = sum(1 for i in range(nreq) if done[i][1]["t_submit_ns"] - int(sched[i]) > 5_000_000)
        search_s = tot["search_ms"] * 1e-3
        lv = {"rho": rho, "requests_per_s": round(lam, 1), "p50_ms": round(percentile(lat, 0.50), 3),
              "p99_ms": round(percentile(lat, 0.99), 3), "served_reads_per_s": round(reads_meas / span, 1),
              "offered_reads_per_s": round(rho * x_off, 1), "failed": sum(1 for v in done.values() if v[0] != 0),
              "submits_late_over_5ms": late,
              # the served search kernels: their device time over all batches
              # (warm-up included), reads per second of it, and bytes touched
              # per second of it against the 8 TB/s peak
              "batches": tot["batches"], "search_ms": round(tot["search_ms"], 3),
              "search_reads_per_s": round(tot["reads"] / search_s, 1) if search_s > 0 else None,
              "search_touched_GBps": round(touched_per_read * tot["reads"] / search_s / 1e9, 2) if search_s > 0 else None,
              "search_touched_frac": round(touched_per_read * tot["reads"] / search_s / 1e9 / HBM_PEAK_GBS, 4)
              if search_s > 0 else None,
              "upload_bytes": tot["upload_bytes"]}
        levels.append(lv)
        log(f"rho={rho}: {lv}")
    line = {
        "metric": METRIC, "value": levels[-1]["served_reads_per_s"], "unit": "reads/s", "n_gpus": 1,
        "steps": len(levels), "warmup": args.serve_warmup, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic (seeded generators, no external data)",
        "config": {"workload": "c5: open-loop Poisson requests over the " + " and ".join(names) + " references, "
                               "1-100,000 reads each (log-uniform), 30-300 bp", "requests_per_level": args.serve_requests,
                   "distinct_requests": args.serve_pool, "batch_linger_us": args.serve_linger_us,
                   "max_batch_reads": args.serve_batch_reads},
        "offline_reads_per_s": round(x_off, 1), "levels": levels,
        "served_touched_bytes_per_read": round(touched_per_read, 1),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
