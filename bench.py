#!/usr/bin/env python3
"""Benchmark of the gfx950 ZipNN codec (byte grouping + chunked Huffman).

Default workload: the synthetic 8B-parameter decoder checkpoint (291 BF16
tensors, 16.06 GB: embedding and head N(0, 0.01), projections N(0, 0.02),
RMSNorm vectors 1 + N(0, 0.05)), batched: every kernel runs once for all
tensors and the decode replays a hipGraph; chunk size and sub-stream length
are picked by the autotuner in 64 KiB .. 1 MiB.

One step = the whole hot path on the checkpoint, inputs resident in HBM:
batched compress (split + histogram + code build + placement + bit packing)
then batched decompress (table build + Huffman decode + merge + store).  The
headline `value` is decode throughput in GB/s of uncompressed bytes (the
paper's convention), from HIP events around every decode launch of the timed
steps (on the stream the graph runs on); `encode_GBps` is the same for
compress.  The same line carries the plain per-tensor decode, the roofline of
the decode kernel, the oracle timed on the host cores (1 thread and up to
16), and a serving block: the continuous-batching server against plain
per-request launches at 100, 1000 and 5000 requests/s plus a closed loop.

Prints ONE JSON line.  `--gpus N` with N > 1 is refused: the codec runs on
one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def _src_hash(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(workload: str, alg_bytes: int):
    """HBM bytes per decode launch from a committed rocprofv3 counter summary
    of this workload (profiles/k_decode_<workload>[_<shape>]_traffic.json)
    taken on the same decoder source and the same containers (equal
    algorithmic bytes, so the same chunk size and S), or None."""
    import glob

    sha = _src_hash(os.path.join(ROOT, "paper_2411_05239_amd", "csrc", "decode.hip"))
    paths = [os.path.join(ROOT, "profiles", f"k_decode_{workload}_traffic.json")]
    paths += sorted(glob.glob(os.path.join(ROOT, "profiles", f"k_decode_{workload}_*_traffic.json")))
    for path in paths:
        try:
            rec = json.load(open(path))
        except Exception:
            continue
        if rec.get("decode_src_sha") == sha and rec.get("algorithmic_bytes_per_launch") == alg_bytes:
            return rec.get("hbm_bytes_per_launch")
    return None


def make_workload(name: str, probe_skip: int = 0, exponent: bool = False):
    import torch

    from paper_2411_05239_amd import workloads
    from paper_2411_05239_amd import zipnn as Z

    if name == "fp32_256mb":
        x = workloads.fp32_rows(8192, 8192, seed=1)
        p = Z.make_params(Z.ZIPNN_FP32, probe_skip=probe_skip, exponent=exponent)
        desc = {"workload": "fp32_8192x8192_rowsigma_loguniform_1e-3_1e-1", "dtype": "fp32", "elements": x.numel(),
                "bytes": x.numel() * 4, "chunk_bytes": p.chunk_bytes, "S": p.substream_syms, "g": p.group,
                "L": p.max_code_len, "policy": "auto", "probe_skip": p.probe_skip, "exponent": p.exponent}
    elif name == "bf16_8mb":
        x = workloads.bf16_normal(4_194_304, seed=0)
        p = Z.make_params(Z.ZIPNN_BF16, policy=[Z.ZIPNN_HUF, Z.ZIPNN_RAW], probe_skip=probe_skip, exponent=exponent)
        desc = {"workload": "bf16_4194304_normal_0.02", "dtype": "bf16", "elements": x.numel(),
                "bytes": x.numel() * 2, "chunk_bytes": p.chunk_bytes, "S": p.substream_syms, "g": p.group,
                "L": p.max_code_len, "policy": "huf,raw", "probe_skip": p.probe_skip, "exponent": p.exponent}
    else:
        raise SystemExit(f"unknown workload {name}")
    return x, p, desc


HOST_THREADS = 16   # at most this many host threads: the CPU share of one GPU on a shared node


def host_info() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def oracle_legs(tensors, bases, p, gpu_containers, budget_s: float, sample: str) -> dict:
    """The oracle (plain C, test infrastructure) on the host cores, at 1
    thread and at one GPU's share of the host threads: every sample tensor is
    compressed once (its container compared with the GPU's) and the sample is
    decompressed repeatedly until `budget_s` seconds of decode have passed."""
    import numpy as np

    import oracle

    from paper_2411_05239_amd import zipnn as Z

    many = max(1, min(HOST_THREADS, os.cpu_count() or 1))
    kw = dict(chunk_bytes=p.chunk_bytes, S=p.substream_syms, g=p.group, L=p.max_code_len, policy=list(p.policy),
              skip=p.probe_skip, exp=bool(p.exponent))
    U = sum(x.numel() * x.element_size() for x in tensors)
    legs, matches, ok = {}, True, True
    for th in (many, 1):
        t_enc, cs = 0.0, []
        for i, x in enumerate(tensors):
            t0 = time.perf_counter()
            c = oracle.compress(x, Z.torch_dtype_code(x.dtype), base=bases[i] if bases else None, nthreads=th, **kw)
            t_enc += time.perf_counter() - t0
            if th == many:
                matches &= bool(np.array_equal(c, gpu_containers[i]))
            cs.append(c)
        reps, t_dec = 0, 0.0
        while reps == 0 or t_dec < budget_s:
            for i, c in enumerate(cs):
                t0 = time.perf_counter()
                d = oracle.decompress(c, base=bases[i] if bases else None, nthreads=th)
                t_dec += time.perf_counter() - t0
                if reps == 0:
                    ok &= bool(np.array_equal(d, oracle.as_bytes(tensors[i])))
            reps += 1
        legs[th] = {"decode_GBps": round(U * reps / t_dec / 1e9, 4), "encode_GBps": round(U / t_enc / 1e9, 4),
                    "threads": th, "decode_passes": reps}
    return {"value": legs[many]["decode_GBps"], "unit": "GB/s", "cores": many, "kind": "oracle",
            "sample": f"{sample} ({U} bytes): 1 compress + {legs[many]['decode_passes']} decompress passes at "
                      f"{many} threads; 1 compress + {legs[1]['decode_passes']} decompress passes at 1 thread",
            "encode_GBps": legs[many]["encode_GBps"], "single_thread": legs[1],
            "host": {**host_info(), "threads_used": many,
                     "note": f"the all-cores leg uses at most {HOST_THREADS} host threads, one GPU's share"},
            "roundtrip_ok": ok, "containers_match_gpu": matches}


def run_single(args):
    import torch

    from paper_2411_05239_amd import zipnn as Z

    x_cpu, p, desc = make_workload(args.workload, args.probe_skip, args.exponent)
    if args.chunk_bytes:
        p.chunk_bytes = args.chunk_bytes
        p.substream_syms = args.substream_syms
        desc.update(chunk_bytes=p.chunk_bytes, S=p.substream_syms)
    dev = torch.device("cuda", 0)
    x = x_cpu.to(dev)
    U = x.numel() * x.element_size()
    codec = Z.Codec(0)
    stream = torch.cuda.current_stream()

    # correctness gate before any number: GPU round trip bit-exact
    c = codec.compress(x, p)
    out = torch.empty_like(x)
    codec.decompress(c, out)
    if not torch.equal(out.view(torch.uint8), x.view(torch.uint8)):
        print(json.dumps({"error": "round trip mismatch"}))
        sys.exit(1)
    C = c.numel()
    hdr = c[:64].cpu().numpy().tobytes()   # host copy of the header: decode launches without a round trip
    cbuf = torch.empty(Z.zipnn_compress_bound(Z.torch_dtype_code(x.dtype), x.numel(), p), dtype=torch.uint8,
                       device=dev)
    scrub = torch.empty(1 << 30, dtype=torch.uint8, device=dev)

    def step(i, timed, ev):
        scrub.fill_(i & 0xFF)   # evict the 256 MB last-level cache between steps
        if not args.decode_only:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            cc = codec.compress(x, p, out=cbuf)
            e1.record(stream)
            assert cc.numel() == C
            ev["enc"].append((e0, e1))
            scrub.fill_((i + 1) & 0xFF)
        d0 = torch.cuda.Event(enable_timing=True)
        d1 = torch.cuda.Event(enable_timing=True)
        d0.record(stream)
        Z.zipnn_decompress_async(codec.ctx, hdr, c.data_ptr(), C, None, out.data_ptr(), U, stream.cuda_stream)
        d1.record(stream)
        ev["dec"].append((d0, d1))

    ev = {"enc": [], "dec": []}
    for i in range(args.warmup):
        step(i, False, ev)
    torch.cuda.synchronize()
    ev = {"enc": [], "dec": []}
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i, True, ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = codec.status()
    if st != Z.ZIPNN_OK or not torch.equal(out.view(torch.uint8), x.view(torch.uint8)):
        print(json.dumps({"error": f"decode status {st} or mismatch after timing"}))
        sys.exit(1)
    # plain device copy of the same byte count: the achievable streaming rate
    # beside the 8 TB/s peak, and the calibration kernel for HBM counters
    cp = []
    for i in range(max(3, args.steps // 2)):
        scrub.fill_(i & 0xFF)
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        out.copy_(x)
        a1.record(stream)
        cp.append((a0, a1))
    torch.cuda.synchronize()
    copy_ms = statistics.median(a.elapsed_time(b) for a, b in cp)
    dec_ms = [a.elapsed_time(b) for a, b in ev["dec"]]
    enc_ms = [a.elapsed_time(b) for a, b in ev["enc"]]
    dec_avg = statistics.mean(dec_ms)
    alg = C + U  # decode: read the container, write the tensor
    achieved = alg / (dec_avg * 1e-3) / 1e9
    traffic = _traffic(args.workload, alg)
    rec = {
        "metric": "decode GB/s at bit-exact roundtrip (uncompressed bytes / decode time); encode GB/s beside it",
        "value": round(U / (dec_avg * 1e-3) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": desc,
        "decode_ms": {"mean": round(dec_avg, 4), "median": round(statistics.median(dec_ms), 4),
                      "p10": round(sorted(dec_ms)[len(dec_ms) // 10], 4),
                      "p90": round(sorted(dec_ms)[(len(dec_ms) * 9) // 10], 4)},
        "encode_GBps": round(U / (statistics.mean(enc_ms) * 1e-3) / 1e9, 2) if enc_ms else None,
        "encode_ms": {"mean": round(statistics.mean(enc_ms), 4), "median": round(statistics.median(enc_ms), 4)}
        if enc_ms else None,
        "compressed_bytes": C,
        "ratio": round(C / U, 5),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": "k_decode", "algorithmic_bytes_per_launch": alg},
        "copy_probe_GBps": round(2 * U / (copy_ms * 1e-3) / 1e9, 1),
        "paper_context": "ZipNN CPU: up to 80 GB/s decompression, 13 GB/s compression (Xeon 8480+, 16 workers)",
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = oracle_legs([x_cpu], None, p, [c.cpu().numpy()], args.cpu_budget, "the whole tensor")
    print(json.dumps(rec))


def _events():
    import torch

    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _modes(arena_np, offs):
    """Map entries per mode over the containers of an arena (host bytes)."""
    from paper_2411_05239_amd import zipnn as Z

    tot = [0, 0, 0, 0]
    for i in range(len(offs) - 1):
        info = Z.zipnn_inspect(arena_np[offs[i]: offs[i + 1]].tobytes())
        for m in range(4):
            tot[m] += info.entries_by_mode[m]
    return dict(zip(["raw", "huf", "rle", "zg"], tot))


def _container(arena_np, off: int):
    """The container at `off` of a host copy of an arena, by its header's size."""
    total = int.from_bytes(arena_np[off + 32: off + 40].tobytes(), "little")
    return arena_np[off: off + total]


def _kind(name: str) -> str:
    return name.split(".")[-1]


def run_checkpoint(args, delta: bool, zg: bool = False):
    """Synthetic 8B decoder checkpoint (291 BF16 tensors, ~16 GB), batched:
    every kernel runs once for all tensors; decode replays a hipGraph.  With
    delta: the fine-tuned copy is stored as the XOR against the base, every
    byte group Huffman-coded (paper §IV-B); with zg as well, AUTO chooses per
    byte group among RAW, RLE, HUF and the zero-aware ZG mode."""
    import torch

    from paper_2411_05239_amd import workloads
    from paper_2411_05239_amd import zipnn as Z

    specs = workloads.checkpoint_8b_specs()
    xs = [workloads.make_tensor(sp, device="cuda") for sp in specs]
    bases = None
    if delta:
        bases = xs
        xs = [workloads.finetune_delta(b, seed=2000 + i) for i, b in enumerate(bases)]
    torch.cuda.synchronize()
    U = sum(x.numel() * 2 for x in xs)
    codec = Z.Codec(0)
    stream = torch.cuda.current_stream()
    if delta and not zg:
        policy = [Z.ZIPNN_HUF, Z.ZIPNN_HUF]   # Huffman on both byte groups (RLE if single-valued)
    else:
        policy = None   # AUTO: RAW / RLE / HUF / ZG per byte group and chunk
    bptr = [b.data_ptr() for b in bases] if delta else [None] * len(xs)
    # chunk size and sub-stream length: the autotuner, over the paper's range
    # around its 256 KB default (64 KiB .. 1 MiB), on a share of every tensor
    if args.chunk_bytes:
        # a fixed shape (profiling runs): no autotuning
        best, table = Z.make_params(Z.ZIPNN_BF16, chunk_bytes=args.chunk_bytes, S=args.substream_syms,
                                    policy=policy), []
    else:
        best, table = Z.tune_checkpoint(codec, xs, bases, policy)
    best.probe_skip = args.probe_skip
    best.exponent = int(args.exponent)
    smp = Z.autotune_sample([x.numel() for x in xs], 2, Z.TUNE_SAMPLE_BYTES, Z.TUNE_MAX_CHUNK)
    comp = {}
    for sp, k in zip(specs, smp):
        c = comp.setdefault(_kind(sp.name), {"tensors": 0, "bytes": 0})
        c["tensors"] += 1
        c["bytes"] += 2 * k
    arena, offs = codec.compress_batch(xs, best, bases)
    outs = [torch.empty_like(x) for x in xs]
    batch = codec.prepare_batch(arena, offs, outs, bases)
    batch.run(check=True)
    torch.cuda.synchronize()
    if not all(torch.equal(o.view(torch.uint8), x.view(torch.uint8)) for o, x in zip(outs, xs)):
        print(json.dumps({"error": "batched round trip mismatch"}))
        sys.exit(1)
    C = offs[-1]
    # the timed encode replays a prepared encoder (descriptors on the device,
    # launches captured in a hipGraph) writing the same arena
    encoder = codec.prepare_encoder(xs, best, bases, arena=arena)
    enc, dec = [], []
    for i in range(args.warmup + args.steps):
        if i == args.warmup:
            torch.cuda.synchronize()
            t_wall = time.perf_counter()
        if not args.decode_only:
            a0, a1 = _events()
            a0.record(stream)
            offs2 = encoder.run()
            a1.record(stream)
            assert offs2 == offs
        b0, b1 = _events()
        b0.record(stream)
        batch.run()
        b1.record(stream)
        if i >= args.warmup:
            if not args.decode_only:
                enc.append((a0, a1))
            dec.append((b0, b1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    st = codec.status()
    if st != Z.ZIPNN_OK or not all(torch.equal(o.view(torch.uint8), x.view(torch.uint8)) for o, x in zip(outs, xs)):
        print(json.dumps({"error": f"status {st} or mismatch after timing"}))
        sys.exit(1)
    # the plain alternative: one decompress launch per tensor on one stream
    a_np = arena[: C].cpu().numpy()
    hdrs = [a_np[offs[i]: offs[i] + 64].tobytes() for i in range(len(xs))]
    per = []
    for r in range(3):
        p0, p1 = _events()
        p0.record(stream)
        for i, x in enumerate(xs):
            if x.numel() == 0:
                continue
            Z.zipnn_decompress_async(codec.ctx, hdrs[i], arena.data_ptr() + offs[i], offs[i + 1] - offs[i],
                                     bptr[i], outs[i].data_ptr(), x.numel() * 2, stream.cuda_stream)
        p1.record(stream)
        per.append((p0, p1))
    torch.cuda.synchronize()
    # plain device copy of 1 GiB: the achievable streaming rate beside the
    # 8 TB/s peak, and the calibration kernel for the HBM counters
    cin = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    cin.fill_(7)
    cout = torch.empty_like(cin)
    cp = []
    for i in range(5):
        c0, c1 = _events()
        c0.record(stream)
        cout.copy_(cin)
        c1.record(stream)
        cp.append((c0, c1))
    torch.cuda.synchronize()
    copy_ms = statistics.median(a.elapsed_time(b) for a, b in cp)
    del cin, cout
    dec_ms = [a.elapsed_time(b) for a, b in dec]
    enc_ms = [a.elapsed_time(b) for a, b in enc]
    per_ms = min(a.elapsed_time(b) for a, b in per[1:])
    dec_avg = statistics.mean(dec_ms)
    alg = C + U + (U if delta else 0)
    achieved = alg / (dec_avg * 1e-3) / 1e9
    enc_alg = U + (U if delta else 0) + C
    name = ("ckpt8b_delta_zg" if zg else "ckpt8b_delta") if delta else "ckpt8b"
    rec = {
        "metric": "decode/encode GB/s at bit-exact roundtrip; batched-serving vs plain p99 latency",
        "value": round(U / (dec_avg * 1e-3) / 1e9, 2),
        "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": ("xor_delta_of_" if delta else "") + "bf16_8b_decoder_checkpoint_291_tensors"
                               + ("_zg" if zg else ""),
                   "tensor_dtype": "bf16", "tensors": len(xs), "bytes": U, "chunk_bytes": best.chunk_bytes,
                   "S": best.substream_syms, "g": best.group, "L": best.max_code_len,
                   "policy": "huf,huf" if delta and not zg else "auto", "probe_skip": best.probe_skip,
                   "exponent": best.exponent, "batched": "encode and decode each a hipGraph replay of one launch per kernel",
                   "step": "batched encode + batched decode" if not args.decode_only else "batched decode"},
        "decode_ms": {"mean": round(dec_avg, 4), "median": round(statistics.median(dec_ms), 4),
                      "p10": round(sorted(dec_ms)[len(dec_ms) // 10], 4),
                      "p90": round(sorted(dec_ms)[(len(dec_ms) * 9) // 10], 4)},
        "encode_GBps": round(U / (statistics.mean(enc_ms) * 1e-3) / 1e9, 2) if enc_ms else None,
        "encode_ms": {"mean": round(statistics.mean(enc_ms), 4)} if enc_ms else None,
        "encode_roofline_frac": round(enc_alg / (statistics.mean(enc_ms) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
        if enc_ms else None,
        "per_tensor_decode": {"launches": sum(1 for x in xs if x.numel()), "ms": round(per_ms, 4),
                              "GBps": round(U / (per_ms * 1e-3) / 1e9, 2)},
        "compressed_bytes": C, "ratio": round(C / U, 5), "entries_by_mode": _modes(a_np, offs),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": _traffic(name, alg),
                     "kernel": "k_decode", "algorithmic_bytes_per_launch": alg},
        "copy_probe_GBps": round(2 * (1 << 30) / (copy_ms * 1e-3) / 1e9, 1),
        "autotune": {"pick": {"chunk_bytes": best.chunk_bytes, "S": best.substream_syms},
                     "rule": "64 KiB..1 MiB chunks x 256..2048 sub-streams on the whole checkpoint; median of 7 "
                             "decodes; ratio within 1%; rates within 2% of the fastest tie; smallest chunk, then "
                             "best ratio",
                     "sample": {"bytes": 2 * sum(smp), "by_kind": comp},
                     "candidates": [{"chunk_bytes": e.params.chunk_bytes, "S": e.params.substream_syms,
                                     "ratio": round(e.ratio, 5), "decode_GBps": round(e.decode_gbps, 1),
                                     "encode_GBps": round(e.encode_gbps, 1)} for e in table]},
        "paper_context": "ZipNN CPU: up to 80 GB/s decompression, 13 GB/s compression (Xeon 8480+, 16 workers)",
    }
    if not args.no_cpu_baseline:
        # a bounded sample: layer 0's nine tensors (every projection kind and both norms) and the final norm
        idx = [i for i, sp in enumerate(specs) if sp.name.startswith("layers.0.") or sp.name == "final_norm"]
        rec["cpu_baseline"] = oracle_legs([xs[i].cpu() for i in idx], [bases[i].cpu() for i in idx] if delta else None,
                                          best, [_container(a_np, offs[i]) for i in idx], args.cpu_budget,
                                          "layer 0 (q, k, v, o, gate, up, down, 2 norms) and the final norm")
    batch.close()
    encoder.close()
    del outs, arena, batch, encoder, xs, bases
    codec.close()
    torch.cuda.empty_cache()
    if not delta and not args.no_serve and not args.decode_only:
        rec["serving"] = serve_block(args, [int(r) for r in args.serve_rates.split(",")])
    print(json.dumps(rec))


def _pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(round(q * (len(v) - 1))))] if v else None


def _serve_pass(Z, srv, handles, sizes, rate, count, seed):
    """Open loop: Poisson arrivals at `rate`; each request names a corpus item
    drawn uniformly.  A submitter thread keeps the schedule; this thread takes
    completions and releases them.  Returns latency stats."""
    import threading

    import torch

    from paper_2411_05239_amd import workloads

    arr = workloads.poisson_arrivals(rate, count, seed)
    it0 = Z.zipnn_server_stats(srv.h).iterations
    g = torch.Generator().manual_seed(seed)
    pick = torch.randint(0, len(handles), (count,), generator=g).tolist()
    t0 = Z.zipnn_clock() + 0.05
    tickets = {}
    lock = threading.Lock()

    def submitter():
        for k in range(count):
            ta = t0 + arr[k]
            wait = ta - Z.zipnn_clock()
            if wait > 5e-4:
                time.sleep(wait - 3e-4)
            while Z.zipnn_clock() < ta:
                pass
            tk = srv.submit(handles[pick[k]], ta)
            with lock:
                tickets[tk] = pick[k]

    th = threading.Thread(target=submitter)
    th.start()
    lat, nbytes, t_last, n_done = [], 0, t0, 0
    ph = {"admit": [], "launch": [], "run": []}
    deadline = time.monotonic() + 120
    while n_done < count and time.monotonic() < deadline:
        tk = srv.next_done(0.5)
        if tk is None:
            continue
        st, _, tm = srv.poll(tk)
        if st != Z.ZIPNN_OK:
            raise SystemExit(f"served request failed: {st}")
        with lock:
            i = tickets.get(tk)
        srv.release(tk)
        lat.append(tm.t_done - tm.t_arrive)
        ph["admit"].append(tm.t_admit - tm.t_arrive)
        ph["launch"].append(tm.t_launch - tm.t_admit)
        ph["run"].append(tm.t_done - tm.t_launch)
        nbytes += sizes[i] if i is not None else 0
        t_last = max(t_last, tm.t_done)
        n_done += 1
    th.join()
    return {"lat": lat, "ph": ph, "bytes": nbytes, "span": t_last - t0,
            "iters": Z.zipnn_server_stats(srv.h).iterations - it0}


def _serve_stats(rate, parts, sizes):
    """Latency and rate statistics over the passes `parts` of one mode."""
    lat = [v for q in parts for v in q["lat"]]
    ph = {k: [v for q in parts for v in q["ph"][k]] for k in parts[0]["ph"]}
    span = sum(q["span"] for q in parts)
    iters = sum(q["iters"] for q in parts)
    return {"rate": rate, "requests": len(lat), "requests_per_iteration": round(len(lat) / max(iters, 1), 3),
            "p50_ms": round(_pct(lat, 0.5) * 1e3, 3),
            "p99_ms": round(_pct(lat, 0.99) * 1e3, 3), "mean_ms": round(statistics.mean(lat) * 1e3, 3),
            "p99_halves_ms": [round(_pct(q["lat"], 0.99) * 1e3, 3) for q in parts],
            "GBps": round(sum(q["bytes"] for q in parts) / span / 1e9, 2),
            "offered_GBps": round(rate * statistics.mean(sizes) / 1e9, 2),
            "p50_phase_ms": {k: round(_pct(v, 0.5) * 1e3, 4) for k, v in ph.items()},
            "p99_phase_ms": {k: round(_pct(v, 0.99) * 1e3, 4) for k, v in ph.items()}}


def run_series(args):
    """Periodic-base storage of an 11-checkpoint training-like run of a
    0.7 GB BF16 decoder (paper §IV-B "Periodic Base"): total compressed
    fraction and the restore time of the checkpoint with the longest chain,
    for standalone storage and for chain / pairs policies with periods 5 and
    10."""
    import torch

    from paper_2411_05239_amd import workloads
    from paper_2411_05239_amd import zipnn as Z
    from paper_2411_05239_amd.series import CheckpointSeries

    specs = workloads.checkpoint_8b_specs(layers=4, hidden=2048, kv=512, ffn=7168, vocab=32000, seed0=5000)
    model = [workloads.make_tensor(sp, device="cuda") for sp in specs]
    steps = 11
    traj = workloads.trajectory(model, steps=steps, seed=5100)
    U = sum(x.numel() * 2 for x in model)
    codec = Z.Codec(0)
    stream = torch.cuda.current_stream()
    res = {}
    for name, period, mode in [("standalone", 1, "pairs"), ("chain_p5", 5, "chain"), ("chain_p10", 10, "chain"),
                               ("pairs_p5", 5, "pairs"), ("pairs_p10", 10, "pairs")]:
        ser = CheckpointSeries(codec, period, mode)
        for ck in traj:
            ser.append(ck)
        total = sum(st.nbytes for st in ser.stored)
        worst = max(range(steps), key=lambda t: len(ser.chain(t)))
        outs = [torch.empty_like(x) for x in traj[worst]]
        times = []
        for r in range(args.warmup + max(2, min(args.steps, 5))):
            a0, a1 = _events()
            a0.record(stream)
            n = ser.restore(worst, outs)
            a1.record(stream)
            torch.cuda.synchronize()
            if r >= args.warmup:
                times.append(a0.elapsed_time(a1))
        if not all(torch.equal(o.view(torch.uint8), x.view(torch.uint8)) for o, x in zip(outs, traj[worst])):
            print(json.dumps({"error": f"series restore mismatch ({name})"}))
            sys.exit(1)
        res[name] = {"fraction": round(total / (steps * U), 5), "worst_checkpoint": worst, "decodes": n,
                     "restore_ms": round(statistics.median(times), 3),
                     "delta_fractions": [round(st.nbytes / U, 4) for st in ser.stored]}
        del ser
        torch.cuda.empty_cache()
    rec = {
        "metric": "periodic-base checkpoint storage: compressed bytes / raw bytes of the whole run",
        "value": res["chain_p10"]["fraction"], "unit": "fraction", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "higher_is_better": False, "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "bf16_0.7gb_decoder_training_run_11_checkpoints", "checkpoint_bytes": U,
                   "trajectory": "p_t = 0.3*0.7^t, sigma_t = 3e-4*0.7^t", "params": "defaults (AUTO, ZG allowed)"},
        "policies": res,
    }
    print(json.dumps(rec))


def serve_block(args, rates) -> dict:
    """Serving loop: a corpus of 128 tensors (64 KiB - 1 GiB log-uniform,
    60/30/10 BF16/FP32/FP8) resident compressed; Poisson request streams at
    `rates` decoded by the continuous-batching server and by the same server
    launching one decode per request; first a closed-loop pass (every item
    requested at once) whose results are checked byte for byte against the
    original tensors."""
    import torch

    from paper_2411_05239_amd import workloads
    from paper_2411_05239_amd import zipnn as Z

    sys.setswitchinterval(2e-4)   # the submitter and the completion threads share the interpreter
    codec = Z.Codec(0)
    items = workloads.serving_corpus()
    xs, cs = [], []
    for it in items:
        x = workloads.make_corpus_tensor(it, device="cuda")
        c = codec.compress(x).clone()
        xs.append(x)
        cs.append(c)
    torch.cuda.synchronize()
    sizes = [x.numel() * x.element_size() for x in xs]
    U, C = sum(sizes), sum(c.numel() for c in cs)
    # one server, switched between the two modes: both use the same output
    # pool, stream and registrations (two servers, one per mode, measured up
    # to 4% apart at low rates, either one ahead, in either creation order)
    res, closed = {}, {}
    modes = {"continuous": Z.ZIPNN_SERVE_CONTINUOUS, "per_request": Z.ZIPNN_SERVE_PER_REQUEST}
    srv = Z.Server(codec, pool_bytes=16 << 30, max_inflight=256, mode=modes["continuous"])
    handles = [srv.register(c) for c in cs]
    for name, mode in modes.items():
        srv.set_mode(mode)
        it0 = Z.zipnn_server_stats(srv.h).iterations
        # closed loop: all items at t=0, every result checked
        t0 = Z.zipnn_clock()
        tks = {srv.submit(h, t0): i for i, h in enumerate(handles)}
        lat, t_last, ok, got = [], t0, True, []
        while len(got) < len(tks):
            tk = srv.next_done(5.0)
            if tk is None:
                raise SystemExit("closed-loop pass stalled")
            st, _, tm = srv.poll(tk)
            ok &= st == Z.ZIPNN_OK
            lat.append(tm.t_done - tm.t_arrive)
            t_last = max(t_last, tm.t_done)
            got.append(tk)
        # every output stays in the pool until checked against the original tensor
        for tk in got:
            i = tks[tk]
            ok &= bool(torch.equal(srv.output(tk, handles[i]), xs[i].contiguous().view(torch.uint8).reshape(-1)))
            srv.release(tk)
        closed[name] = {"requests": len(tks), "seconds": round(t_last - t0, 4),
                        "GBps": round(U / (t_last - t0) / 1e9, 2), "p50_ms": round(_pct(lat, 0.5) * 1e3, 3),
                        "p99_ms": round(_pct(lat, 0.99) * 1e3, 3), "all_equal_original": ok}
        closed[name]["iterations"] = Z.zipnn_server_stats(srv.h).iterations - it0
    # open loop: per rate two halves of the same two request streams, run
    # continuous, per-request, per-request, continuous, so that neither mode
    # gains from going second; at least 1000 requests per rate and mode, so
    # that p99 is the 10th slowest, not the 2nd
    res = {"continuous": [], "per_request": []}
    for ri, rate in enumerate(rates):
        half = int(min(2000, max(500, rate * args.serve_seconds / 2)))
        parts = {"continuous": [], "per_request": []}
        for name, h in (("continuous", 0), ("per_request", 0), ("per_request", 1), ("continuous", 1)):
            srv.set_mode(modes[name])
            parts[name].append(_serve_pass(Z, srv, handles, sizes, rate, half, 4000 + 2 * ri + h))
        for name in res:
            res[name].append(_serve_stats(rate, parts[name], sizes))
            print(json.dumps({"progress": name, **res[name][-1]}), file=sys.stderr, flush=True)
    srv.close()
    codec.close()
    del xs, cs
    torch.cuda.empty_cache()
    # where continuous batching finds no second request to join an iteration
    # (requests_per_iteration near 1), both modes launch the same
    # iterations, one request each, and their p99s differ by run-to-run noise:
    # the gap is set beside the spread of one mode's p99 between its two halves
    def spread(r):
        return max(r["p99_halves_ms"]) - min(r["p99_halves_ms"])

    cmp = [{"rate": a["rate"], "p99_continuous_ms": a["p99_ms"], "p99_per_request_ms": b["p99_ms"],
            "continuous_p99_le_per_request": a["p99_ms"] <= b["p99_ms"],
            "p99_ratio": round(a["p99_ms"] / b["p99_ms"], 4) if b["p99_ms"] else None,
            "p99_gap_ms": round(a["p99_ms"] - b["p99_ms"], 3),
            "p99_half_to_half_spread_ms": round(max(spread(a), spread(b)), 3),
            "requests_per_iteration_continuous": a["requests_per_iteration"],
            "GBps_continuous": a["GBps"], "GBps_per_request": b["GBps"]}
           for a, b in zip(res["continuous"], res["per_request"])]
    return {"workload": "serving_corpus_128_tensors_64KiB_1GiB_bf16_fp32_fp8", "bytes": U, "compressed_bytes": C,
            "pool_bytes": 16 << 30, "rates": rates, "closed_loop": closed, "open_loop": res, "comparison": cmp}


def run_serve(args):
    """The serving loop alone, over the full rate sweep (100 - 5000/s)."""
    rates = [100, 200, 500, 1000, 2000, 5000]
    blk = serve_block(args, rates)
    cl = blk["closed_loop"]["continuous"]
    alg = blk["compressed_bytes"] + blk["bytes"]
    rec = {
        "metric": "decode/encode GB/s at bit-exact roundtrip; batched-serving vs plain p99 latency",
        "value": cl["GBps"], "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(cl["seconds"] * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": blk["workload"], "bytes": blk["bytes"], "compressed_bytes": blk["compressed_bytes"],
                   "pool_bytes": blk["pool_bytes"], "chunks_per_iter": 2048, "rates": rates},
        "closed_loop": blk["closed_loop"], "open_loop": blk["open_loop"], "comparison": blk["comparison"],
        "roofline": {"bound": "hbm", "achieved": round(alg / cl["seconds"] / 1e9, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(alg / cl["seconds"] / 1e9 / HBM_PEAK_GBPS, 4), "traffic": None,
                     "kernel": "k_decode (server iterations; wall clock of the closed-loop pass)",
                     "algorithmic_bytes_per_launch": alg},
    }
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ckpt8b",
                    choices=["bf16_8mb", "fp32_256mb", "ckpt8b", "ckpt8b_delta", "ckpt8b_delta_zg", "serve",
                             "series"])
    ap.add_argument("--serve-seconds", type=float, default=1.0, help="seconds of arrivals per rate")
    ap.add_argument("--serve-rates", default="100,1000,5000", help="ckpt8b: rates of the serving block")
    ap.add_argument("--no-serve", action="store_true", help="ckpt8b: leave out the serving block")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=4.0, help="seconds of oracle decode per thread count")
    ap.add_argument("--decode-only", action="store_true", help="time decode launches only (for profiling)")
    ap.add_argument("--exponent", action="store_true",
                    help="exponent extraction (BF16 / FP32): the exponent byte is exactly the 8 exponent bits")
    ap.add_argument("--chunk-bytes", type=int, default=0,
                    help="checkpoint workloads: use this chunk size (with --substream-syms) instead of autotuning")
    ap.add_argument("--substream-syms", type=int, default=None, help="S with --chunk-bytes")
    ap.add_argument("--probe-skip", type=int, default=0,
                    help="compressibility probing interval K (0: off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the codec runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "serve":
        run_serve(args)
    elif args.workload in ("ckpt8b", "ckpt8b_delta", "ckpt8b_delta_zg"):
        run_checkpoint(args, delta=args.workload != "ckpt8b", zg=args.workload == "ckpt8b_delta_zg")
    elif args.workload == "series":
        run_series(args)
    else:
        run_single(args)


if __name__ == "__main__":
    main()
