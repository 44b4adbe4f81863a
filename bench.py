"""Benchmark of the DDGI-resampling hot path on one MI355X.

A step is one frame of the 1920x1080 workload (room with 128 spheres + 128
boxes, 32x8x32 probes, M=32 candidates, temporal reuse, two spatial passes
with k=5 and radius 30 px): G-buffer, initial resampling, temporal reuse,
two spatial passes and shading, with all inputs resident in HBM.  The probe
volume is filled before the timed region (the workload updates it only
before frame 0).

Prints one JSON line: resampled pixels per second over whole frames, the
per-kernel HIP-event times, the roofline of the dominant kernel, the same
frame with the learned cache as the target (BF16 and FP8 inference, online
BF16 training; speed ratio to the probe form and the MFMA roofline of the
inference kernel) and the FP64 oracle's rate on a bounded crop of the same
frame (CPU baseline).
"""
import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per pixel each pass must move through HBM with this
# layout (16-byte G-buffer and reservoir records; padding lanes excluded):
#   gbuffer  writes pos+depth 16, normal+prim 16, albedo 12, emit 12 = 56
#   initial  reads x, n, rho (12+12+12 = 36); writes reservoir 56 + resid 12 = 104
#   temporal reads G-buffer 40 + current reservoir 56 + history 56 + prev G-buffer 28
#            = 180 (+ writes 56) = 236
#   spatial  reads G-buffer 40 + own reservoir 56; writes 56 = 152 (neighbour
#            records are re-reads of the same buffer)
#   shade    reads G-buffer 52 + reservoir 56 + resid 12; writes 12 = 132
ALGO_BYTES = {"gbuffer": 56, "initial": 104, "temporal": 236, "spatial": 152, "shade": 132}
# learned-cache training options set from the command line (empty: the binding's defaults)
MLP_OPTS = {}
# probe-record bytes one probe fetch reads (irradiance + depth quad) per texel format
PROBE_RECORD_BYTES = {"f32": 48 + 32, "f16": 24 + 16}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="hd")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-crop", type=int, nargs=2, default=(320, 180))
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-cache forms")
    ap.add_argument("--probe-texel", choices=["f32", "f16"], default="f32",
                    help="probe texel storage of the timed probe form (the workloads specify FP32)")
    ap.add_argument("--no-f16-form", action="store_true",
                    help="skip the extra timing of the same frames from binary16 probe textures")
    ap.add_argument("--mlp-train-frames", type=int, default=64,
                    help="untimed frames of online training before the learned-cache forms are timed")
    ap.add_argument("--mlp-ema", type=float, default=None,
                    help="decay of the parameter average the cache's inference uses (default: the binding's)")
    ap.add_argument("--mlp-steps", type=int, default=None,
                    help="Adam steps per frame over the frame's training batch (default: the binding's)")
    ap.add_argument("--mlp-only", choices=["bf16", "fp8"], default=None,
                    help="time only this learned-cache form (for profiling)")
    ap.add_argument("--quality", action="store_true",
                    help="instead of timing: image MSE of the probe and learned-cache forms against "
                         "path-traced references (prints one JSON line)")
    ap.add_argument("--quality-frames", type=int, default=64)
    ap.add_argument("--quality-eval", type=int, default=32, help="last frames scored")
    ap.add_argument("--quality-seeds", type=int, default=2, help="render seeds averaged")
    ap.add_argument("--ref-spp", type=int, default=2048)
    ap.add_argument("--profile-copy", action="store_true",
                    help="after the timed region, copy 1 GiB device-to-device once (a known-size "
                         "reference for the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--profile-commands", metavar="DIR", default=None,
                    help="print the rocprofv3 commands behind profiles/ (results under DIR) and exit")
    ap.add_argument("--summarize-profiles", metavar="DIR", default=None,
                    help="write the profiles/ summaries from those runs' results under DIR and exit")
    return ap.parse_args()


# sources a committed profile depends on: the resampling kernels, or the learned cache's
KERNEL_SOURCES = {
    "resampling": ["paper_2108_05263_amd/csrc/gi_kernels.hip", "paper_2108_05263_amd/csrc/gi_device.hpp",
                   "include/gi.h"],
    "mlp": ["paper_2108_05263_amd/csrc/gi_mlp.hip", "paper_2108_05263_amd/csrc/gi_mlp.hpp",
            "paper_2108_05263_amd/csrc/gi_device.hpp", "include/gi.h"],
}


def source_sha(family="resampling"):
    """SHA-256 prefix of the kernel sources of one family (profiles record it)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile(kernel, workload, what):
    """A committed rocprofv3 counter summary (profiles/<kernel>_<workload>_<what>.json)
    if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{what}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != source_sha("mlp" if kernel.startswith("k_mlp") else "resampling"):
        return None
    return rec


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the FETCH_SIZE / WRITE_SIZE runs."""
    rec = _profile(kernel, workload, "traffic")
    return None if rec is None else rec.get("traffic_bytes_per_launch")


# Vector-ALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction
# per SIMD every 4 cycles (16 lanes per cycle; packed FP32 is not used).
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4


def alu_issue(kernel, workload, ms):
    """Measured vector-ALU issue rate of `kernel`: its VALU wave-instructions
    per launch (SQ_INSTS_VALU from the committed counter run) over the live
    launch time, against the issue peak."""
    rec = _profile(kernel, workload, "sq_counters")
    if rec is None:
        return None
    insts = rec["SQ_INSTS_VALU"]
    achieved = insts / (ms * 1e-3) / 1e9
    return {"valu_insts_per_launch": insts, "achieved": achieved, "peak": VALU_PEAK_GINST,
            "unit": "G wave-instr/s", "frac": achieved / VALU_PEAK_GINST,
            "source": f"profiles/{kernel}_{workload}_sq_counters.json"}


def _host():
    """Host CPU: model name, logical CPUs, CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def _oracle_frame(o, sg, cfg, sc, grid, irr, dep, pix, f, prev=None):
    """One frame of the oracle on the listed pixels (all pixels: None); per-pass
    seconds.  prev = (G-buffer, history reservoirs, camera) of the frame before."""
    import numpy as np
    W, H = cfg.width, cfg.height
    pr = cfg.params
    cam = sg.make_camera(cfg, f)
    t = {}
    t0 = time.perf_counter()
    gb = o.gbuffer(sc, cam, pixels=pix, out=np.zeros((W * H, 14)) if pix is not None else None)
    t["gbuffer"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    res, resid = o.resample_initial(sc, W, H, gb, grid, irr, dep, pr, 1, f, pixels=pix)
    t["initial"] = time.perf_counter() - t0
    if prev is not None and pr.temporal:
        t0 = time.perf_counter()
        res = o.resample_temporal(sc, W, H, gb, prev[0], prev[2], res, prev[1], pr, 1, f, pixels=pix)
        t["temporal"] = time.perf_counter() - t0
    for sp in range(pr.n_spatial):
        t0 = time.perf_counter()
        res = o.resample_spatial(sc, W, H, gb, res, pr, sp, 1, f, pixels=pix)
        t[f"spatial{sp}"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.shade(sc, W, H, gb, grid, irr, dep, res, resid, pr, pixels=pix)
    t["shade"] = time.perf_counter() - t0
    return t, (gb, res, cam)


def cpu_baseline(cfg, crop):
    """The FP64 oracle on the host: the 1920x1080 workload's frame 0 in full on
    the oracle's OpenMP pixel loops (all usable CPUs, at most 16: the host share
    of one GPU), the 64x64 room's frame in full on one thread, and a centred
    crop of the 1920x1080 workload's second frame (with temporal reuse) on one
    thread.  The probe volume is filled once beforehand with fewer rays (it is
    an input of the timed passes, not timed)."""
    import numpy as np
    import oracle as o
    from paper_2108_05263_amd import scenegen as sg

    host = _host()
    threads = o.set_threads(min(16, host["usable_cpus"] or 1))
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    irr, dep = o.fill_probes(sc, grid, sg.ProbeUpdate(rays=32, fill_passes=1, fill_rays=32), seed=1)
    W, H = cfg.width, cfg.height
    tf, _ = _oracle_frame(o, sg, cfg, sc, grid, irr, dep, None, 0)
    full_s = sum(tf.values())
    o.set_threads(1)
    # the 64x64 room, one frame in full, one thread
    tcfg = sg.CONFIGS["tiny"]
    tsc, tgrid = sg.make_scene(tcfg), sg.make_probe_grid(tcfg)
    tirr, tdep = o.fill_probes(tsc, tgrid, tcfg.probe_update, seed=1)
    tt, _ = _oracle_frame(o, sg, tcfg, tsc, tgrid, tirr, tdep, None, 0)
    tiny_s = sum(tt.values())
    # single-thread rate on the 1080p frame: a centred crop of frame 1 (temporal reuse on)
    cw, ch = crop
    x0, y0 = (W - cw) // 2, (H - ch) // 2
    pix = np.array([(y0 + j) * W + x0 + i for j in range(ch) for i in range(cw)], np.int32)
    _, prev = _oracle_frame(o, sg, cfg, sc, grid, irr, dep, pix, 0)
    tc, _ = _oracle_frame(o, sg, cfg, sc, grid, irr, dep, pix, 1, prev)
    crop_s = sum(tc.values())
    return {"value": W * H / full_s, "unit": "pixels/s", "cores": threads, "kind": "oracle",
            "sample": f"{W}x{H} workload, frame 0 in full (G-buffer, initial, {cfg.params.n_spatial} spatial "
                      f"passes, shading; no temporal pass in frame 0), FP64, {threads} OpenMP threads, "
                      f"{full_s:.1f} s",
            "pass_s": {k: round(v, 3) for k, v in tf.items()},
            "host": host,
            "single_thread": {
                "tiny_64x64_frame_s": round(tiny_s, 3), "tiny_pixels_per_s": 64 * 64 / tiny_s,
                "hd_crop": f"{cw}x{ch} centre crop of frame 1 (with temporal reuse)",
                "hd_crop_pixels_per_s": len(pix) / crop_s, "hd_crop_s": round(crop_s, 3)}}


# Algorithmic FLOP of one network evaluation: 2 * (78*64 + 3*64*64 + 64*3)
MLP_FLOP = 34944
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0}


def mlp_form(gi, sg, torch, cfg, precision, steps, warmup, mode="always", train_frames=0):
    """Frames of the learned-cache form (cache target in the initial pass and
    in shading, online training after each frame), timed like the probe form,
    plus the inference kernel alone on one frame's candidates.  mode "always"
    makes the cache the target in every frame; "auto" lets the cache's own
    judge (its error against the probe query) decide per frame, falling back
    to the probe query.  train_frames untimed frames of online training run
    before the warm-up (the cache in steady state)."""
    r = gi.Renderer(cfg, seed=1, mlp=precision, mlp_mode=mode, **MLP_OPTS)
    r.fill_probes()
    stream = torch.cuda.current_stream()
    keys = {"trace_gbuffer": "gbuffer", "resample_initial_mlp": "initial", "resample_temporal": "temporal",
            "shade_mlp": "shade", "mlp_make_batch": "batch"}
    orig = {k: getattr(gi, k) for k in list(keys) + ["resample_spatial"]}
    pending = []

    def timed(key_fn, fn):
        def wrapper(*a, **kw):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn(*a, **kw)
            e1.record(stream)
            pending.append((key_fn(a), e0, e1))
        return wrapper

    for k, name in keys.items():
        setattr(gi, k, timed(lambda a, name=name: name, orig[k]))
    gi.resample_spatial = timed(lambda a: f"spatial{a[4]}", orig["resample_spatial"])
    orig_train = r.train_mlp
    r.train_mlp = timed(lambda a: "train", orig_train)
    try:
        f0 = train_frames + warmup
        for f in range(f0):
            r.frame(f)
        torch.cuda.synchronize()
        pending.clear()
        t0 = time.perf_counter()
        for f in range(f0, f0 + steps):
            r.frame(f)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    finally:
        for k, v in orig.items():
            setattr(gi, k, v)
    times = {}
    for key, e0, e1 in pending:
        times.setdefault(key, []).append(e0.elapsed_time(e1))
    avg = {k: sum(v) / len(v) for k, v in times.items()}
    st = r.mlp.state_words()
    # inference alone on the last frame's candidate points (M per pixel)
    n = r.W * r.H * r.params.M
    ws = r.ws_init.view(torch.float32).view(-1, 4)
    pos, nrm = ws[:n], ws[n:2 * n]
    out = torch.empty(n, 4, dtype=torch.float32, device="cuda")
    lib = gi.load()
    import ctypes as C

    def infer():
        gi.check(lib.gi_mlp_infer(r.mlp.ref, n, C.c_void_p(pos.data_ptr()), C.c_void_p(nrm.data_ptr()),
                                  C.c_void_p(out.data_ptr()), C.c_void_p(stream.cuda_stream)), "gi_mlp_infer")
    infer()
    torch.cuda.synchronize()
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        infer()
    e1.record(stream)
    torch.cuda.synchronize()
    t_inf = e0.elapsed_time(e1) / reps
    tflops = n * MLP_FLOP / (t_inf * 1e-3) / 1e12
    npx = r.W * r.H
    res_ms = sum(v for k, v in avg.items() if k not in ("gbuffer", "batch", "train"))
    return {
        "mode": mode,
        "trained_frames_before_timing": f0,
        "ms_per_step": elapsed * 1e3 / steps,
        "pixels_per_s": npx * steps / elapsed,
        "resampling_only_pixels_per_s": npx / (res_ms * 1e-3),
        "kernel_ms": {k: round(v, 4) for k, v in avg.items()},
        "train": {"samples_per_frame": r.batch.n, "adam_steps_per_frame": r.mlp_steps,
                  "loss": st["loss"], "ema_sq_err_ratio_vs_probe": st["ema_err"], "usable": st["usable"]},
        "infer_kernel": {"samples": n, "ms": t_inf, "bound": "mfma", "achieved": tflops,
                         "peak": MFMA_PEAK_TFLOPS[precision], "unit": "TFLOP/s",
                         "frac": tflops / MFMA_PEAK_TFLOPS[precision], "flop_per_sample": MLP_FLOP},
    }


def reference_image(gi, torch, r, gb, spp, seed, chunk=32):
    """Mean of spp path-traced samples per pixel, in launches of `chunk` samples."""
    acc = torch.zeros(r.W * r.H, 4, dtype=torch.float32, device="cuda")
    tmp = torch.empty_like(acc)
    s0 = 0
    while s0 < spp:
        n = min(chunk, spp - s0)
        gi.path_trace(r.dscene, gb, n, seed, s0, tmp)
        acc += tmp * n
        s0 += n
    return acc[:, :3] / spp


def quality(gi, sg, torch, cfg, frames, n_eval, ref_spp, n_seeds):
    """Frames 0..frames-1 of each form (probe target from FP32 and from
    binary16 texels; learned cache in BF16 / FP8, always the target, trained
    online from frame 0) for render seeds
    1..n_seeds; the last n_eval frames are scored against path-traced
    references of the same camera: MSE over pixels and channels, relative
    MSE (err^2 / (ref^2 + 0.01)) and MAPE (|err| / (ref + 0.01)), averaged
    over frames and seeds.  The reference's own noise is estimated from two
    independent halves (MSE(a, b) / 4 is the expected squared error of their
    mean); it adds the same amount to every form's MSE."""
    eval_frames = list(range(frames - n_eval, frames))
    base = gi.Renderer(cfg, seed=1)
    refs, noise = {}, []
    half = ref_spp // 2
    for f in eval_frames:
        gi.trace_gbuffer(base.dscene, base.camera(f), base.gb[0])
        a = reference_image(gi, torch, base, base.gb[0], half, 777)
        b = reference_image(gi, torch, base, base.gb[0], half, 778)
        refs[f] = (a + b) * 0.5
        noise.append(float(((a - b) ** 2).mean()) / 4.0)
        print(f"reference frame {f} done", file=sys.stderr, flush=True)
    del base
    out = {"config": cfg.name, "frames": frames, "eval_frames": [eval_frames[0], eval_frames[-1]],
           "seeds": n_seeds, "ref_spp": ref_spp, "ref_noise_mse": sum(noise) / len(noise),
           "mlp_options": dict(MLP_OPTS), "forms": {}}
    forms = (("probe", None, "f32"), ("bf16", "bf16", "f32"), ("fp8", "fp8", "f32"))
    if cfg.name == "uhd":
        # the precision sweep: half-precision G-buffer normals and albedo, alone and with FP8 inference
        forms += (("probe, f16 G-buffer", None, "f16"), ("fp8, f16 G-buffer", "fp8", "f16"))
    forms = tuple((name, mlp, gbf, cfg) for name, mlp, gbf in forms)
    # storage precision of the probe textures: the same probe target from binary16 texels
    forms += (("probe, binary16 texels", None, "f32", dataclasses.replace(cfg, probe_texel="f16")),)
    if cfg.glossy_frac > 0.0:
        # glossy workload: the specular recursion of shading at the workload's threshold,
        # switched off (c = 0: every glossy sample read from the probes) and deeper (c = 1);
        # the learned cache serves Lambertian scenes only
        def with_c(c):
            return dataclasses.replace(cfg, params=dataclasses.replace(cfg.params, foot_c=c))
        forms = ((f"probe, recursion c={cfg.params.foot_c:g}", None, "f32", cfg),
                 ("probe, no recursion (c=0)", None, "f32", with_c(0.0)),
                 ("probe, recursion c=1", None, "f32", with_c(1.0)))
    for form, mlp, gbf, fcfg in forms:
        acc = {"mse": [], "relmse": [], "mape": []}
        per_seed, train = [], []
        # per evaluated frame: sum and sum of squares of the image over seeds, to
        # split the error into the squared bias of the seed mean and the variance
        s1 = {f: torch.zeros_like(refs[f]) for f in eval_frames}
        s2 = {f: torch.zeros_like(refs[f]) for f in eval_frames}
        for seed in range(1, n_seeds + 1):
            r = gi.Renderer(fcfg, seed=seed, mlp=mlp, mlp_mode="always", gb_format=gbf,
                            **(MLP_OPTS if mlp is not None else {}))
            r.fill_probes()
            m = {"mse": 0.0, "relmse": 0.0, "mape": 0.0}
            for f in range(frames):
                r.frame(f)
                if f in refs:
                    img = r.img[:, :3]
                    s1[f] += img
                    s2[f] += img * img
                    d = img - refs[f]
                    m["mse"] += float((d * d).mean()) / n_eval
                    m["relmse"] += float((d * d / (refs[f] ** 2 + 1e-2)).mean()) / n_eval
                    m["mape"] += float((d.abs() / (refs[f] + 1e-2)).mean()) / n_eval
            for k in acc:
                acc[k].append(m[k])
            per_seed.append(m["mse"])
            if mlp is not None:
                st = r.mlp.state_words()
                train.append({"loss": st["loss"], "ema_sq_err_ratio_vs_probe": st["ema_err"], "usable": st["usable"]})
            del r
            torch.cuda.empty_cache()
        rec = {k: sum(v) / len(v) for k, v in acc.items()}
        rec["mse_per_seed"] = per_seed
        if n_seeds >= 2:
            # squared bias of the per-frame seed mean: its squared error minus the
            # variance it still carries (sample variance / n_seeds) and the
            # reference's own noise; plus the mean signed error (brightness bias)
            b2, me = 0.0, 0.0
            for f in eval_frames:
                mean = s1[f] / n_seeds
                var = (s2[f] - n_seeds * mean * mean) / (n_seeds - 1)
                b2 += float(((mean - refs[f]) ** 2).mean() - var.mean() / n_seeds) / n_eval
                me += float((mean - refs[f]).mean()) / n_eval
            rec["bias2"] = b2 - out["ref_noise_mse"]
            rec["variance"] = rec["mse"] - b2
            rec["mean_signed_err"] = me
        if train:
            rec["train_at_end"] = train
        out["forms"][form] = rec
        print(f"form {form}: {rec}", file=sys.stderr, flush=True)
    return out


# --------------------------------------------------------------------------
# rocprofv3 runs behind the committed profiles/ summaries
# --------------------------------------------------------------------------
PROBE_INITIAL = "k_initial<true, false, false, false, 0>"    # the probe form's initial pass (scene in LDS, FP32 texels)
# the probe form's other resampling kernels of the 1080p workload (scene in LDS, FP32 texels)
REUSE_KERNELS = ("k_temporal<true, false>", "k_spatial<true, false, 5>", "k_shade<true, false, false, 0>")
SQ_SETS = {"sq1": "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU "
                  "SQ_ACTIVE_INST_LDS SQ_INSTS_VMEM_RD",
           "sq2": "SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_ACTIVE_INST_ANY SQ_THREAD_CYCLES_VALU TCC_HIT_sum "
                  "TCC_MISS_sum GRBM_GUI_ACTIVE"}
MFMA_SET = ("SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CYCLES SQ_INSTS_VALU SQ_INSTS_MFMA SQ_VALU_MFMA_COEXEC_CYCLES "
            "GRBM_GUI_ACTIVE")


def profile_commands(outdir):
    """The rocprofv3 runs (one shell command each) whose results
    summarize_profiles() turns into profiles/: kernel-trace statistics of
    the default benchmark, HBM traffic (FETCH_SIZE, then WRITE_SIZE, each
    scaled by a 1 GiB copy in the same run), SQ counters of the probe form's
    initial pass, MFMA counters of the inference kernels."""
    bench = f"python3 -u {os.path.join(ROOT, 'bench.py')}"
    pre = "cd /tmp && TMPDIR=/tmp timeout -s KILL 240 rocprofv3"
    probe = f"{bench} --steps 2 --warmup 1 --no-cpu --no-mlp --no-f16-form"
    cmds = {"kt": f"{pre} --kernel-trace --stats --output-format csv -d {outdir}/kt -o hd -- "
                  f"{bench} --steps 5 --warmup 2 --no-cpu --mlp-train-frames 8",
            "fetch": f"{pre} --pmc FETCH_SIZE --output-format csv -d {outdir}/fetch -o hd -- {probe} --profile-copy",
            "write": f"{pre} --pmc WRITE_SIZE --output-format csv -d {outdir}/write -o hd -- {probe} --profile-copy"}
    for k, v in SQ_SETS.items():
        cmds[k] = f"{pre} --pmc {v} --output-format csv -d {outdir}/{k} -o hd -- {probe}"
    for prec in ("bf16", "fp8"):
        cmds[f"mfma_{prec}"] = (f"{pre} --pmc {MFMA_SET} --output-format csv -d {outdir}/mfma_{prec} -o mlp -- "
                                f"{bench} --mlp-only {prec} --steps 2 --warmup 1 --mlp-train-frames 0")
    return cmds


def _csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _counters(d, kernel_sub):
    """Per-dispatch counter values (summed over the chip) of the dispatches
    whose kernel name contains kernel_sub: {counter: [value per dispatch]}."""
    per = {}
    for r in _csv_rows(d, "counter_collection.csv"):
        if kernel_sub not in r["Kernel_Name"]:
            continue
        key = (r["Dispatch_Id"], r["Counter_Name"])
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (_, c), v in sorted(per.items(), key=lambda kv: int(kv[0][0])):
        out.setdefault(c, []).append(v)
    return out


def _short(name):
    """Kernel name without namespace, parameter list and return type."""
    n = name.replace("(anonymous namespace)::", "").replace("void ", "", 1)
    return n.split("(")[0].strip()


def summarize_profiles(outdir, ms_initial=None):
    """Write the profiles/ summaries from the runs of profile_commands()."""
    cmds = {k: v.replace(ROOT, "<repo>").replace(outdir, "<out>") for k, v in profile_commands(outdir).items()}
    prof = os.path.join(ROOT, "profiles")
    sha_r, sha_m = source_sha("resampling"), source_sha("mlp")
    written = []
    # kernel-trace statistics
    rows = _csv_rows(os.path.join(outdir, "kt"), "kernel_stats.csv")
    if rows:
        for fname, fam, keep in (("k_initial_hd_kernel_stats.txt", "resampling", lambda n: "k_mlp" not in n),
                                 ("k_mlp_infer_hd_kernel_stats.txt", "mlp", lambda n: "k_mlp" in n or "k_cand" in n)):
            lines = [f"# rocprofv3 kernel-trace statistics, 1920x1080 workload (hd), {fam} kernels of the run",
                     f"# command: {cmds['kt']}",
                     f"# kernel sources: {source_sha(fam)} (sha256 prefix of {', '.join(KERNEL_SOURCES[fam])})",
                     "# the run covers the probe form and the learned-cache forms (BF16, FP8; always and auto)",
                     "# columns: kernel, calls, average ns, min ns, max ns, total ns"]
            for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
                if keep(r["Name"]):
                    lines.append(f'{_short(r["Name"])}, {r["Calls"]}, {float(r["AverageNs"]):.0f}, '
                                 f'{float(r["MinNs"]):.0f}, {float(r["MaxNs"]):.0f}, {float(r["TotalDurationNs"]):.0f}')
            with open(os.path.join(prof, fname), "w") as fh:
                fh.write("\n".join(lines) + "\n")
            written.append(fname)
    # HBM traffic of the probe form's initial pass, scaled by the copy reference
    fetch = _counters(os.path.join(outdir, "fetch"), PROBE_INITIAL).get("FETCH_SIZE", [])
    write = _counters(os.path.join(outdir, "write"), PROBE_INITIAL).get("WRITE_SIZE", [])
    cf = _counters(os.path.join(outdir, "fetch"), "copyBuffer").get("FETCH_SIZE", [])
    cw = _counters(os.path.join(outdir, "write"), "copyBuffer").get("WRITE_SIZE", [])
    if fetch and write and cf and cw:
        gib = float(1 << 30)
        fs, ws = gib / (max(cf) * 1024.0), gib / (max(cw) * 1024.0)
        f_kib, w_kib = sum(fetch) / len(fetch), sum(write) / len(write)
        rec = {"kernel": "k_initial", "workload": "hd 1920x1080, M=32", "source_sha": sha_r,
               "fetch_size_kib_per_dispatch": f_kib, "write_size_kib_per_dispatch": w_kib,
               "dispatches": [len(fetch), len(write)],
               "copy_reference": {"bytes": int(gib), "fetch_size_kib": max(cf), "write_size_kib": max(cw),
                                  "fetch_scale": fs, "write_scale": ws},
               "traffic_bytes_per_launch": int(f_kib * 1024 * fs + w_kib * 1024 * ws),
               "algorithmic_bytes_per_launch": ALGO_BYTES["initial"] * 1920 * 1080,
               "commands": [cmds["fetch"], cmds["write"]],
               "note": "FETCH_SIZE/WRITE_SIZE count L2-to-fabric bytes (MALL or HBM); each is scaled by what "
                       "the same counter reads for a 1 GiB device-to-device copy in the same run"}
        with open(os.path.join(prof, "k_initial_hd_traffic.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        written.append("k_initial_hd_traffic.json")
    # SQ counters of the probe form's initial pass
    rec = {"kernel": "k_initial", "workload": "hd", "source_sha": sha_r}
    for k in SQ_SETS:
        for c, v in _counters(os.path.join(outdir, k), PROBE_INITIAL).items():
            rec[c] = sum(v) / len(v)
            rec[c + "_dispatches"] = len(v)
    if "SQ_INSTS_VALU" in rec:
        rec["commands"] = [cmds[k] for k in SQ_SETS]
        rec["note"] = ("per-dispatch averages summed over the chip; the SQ_*CYCLES / SQ_WAIT* / SQ_ACTIVE* counters "
                       "count quad-cycles (4 clocks), SQ_INSTS_* count wave-level instructions")
        if "SQ_THREAD_CYCLES_VALU" in rec and "SQ_ACTIVE_INST_VALU" in rec:
            rec["active_lanes_per_valu_instruction"] = rec["SQ_THREAD_CYCLES_VALU"] / rec["SQ_ACTIVE_INST_VALU"]
        if "TCC_HIT_sum" in rec:
            rec["l2_hit_rate"] = rec["TCC_HIT_sum"] / (rec["TCC_HIT_sum"] + rec["TCC_MISS_sum"])
        with open(os.path.join(prof, "k_initial_hd_sq_counters.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        written.append("k_initial_hd_sq_counters.json")
    # SQ counters of the reuse passes and shading from the same runs (what bounds them)
    kt_avg = {}
    for r in _csv_rows(os.path.join(outdir, "kt"), "kernel_stats.csv"):
        kt_avg[_short(r["Name"])] = float(r["AverageNs"]) * 1e-6
    reuse = {"kernel_sources": sha_r, "workload": "hd 1920x1080, FP32 probe texels",
             "commands": [cmds[k] for k in SQ_SETS],
             "note": "per-dispatch averages summed over the chip; issue fraction = SQ_INSTS_VALU over the "
                     "kernel-trace average duration x 614.4 G wave-instructions/s; active lanes = "
                     "SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU", "kernels": {}}
    for kname in REUSE_KERNELS:
        rec_k = {}
        for k in SQ_SETS:
            for c, v in _counters(os.path.join(outdir, k), kname).items():
                rec_k[c] = sum(v) / len(v)
        if "SQ_INSTS_VALU" not in rec_k:
            continue
        ms = kt_avg.get(kname)
        if ms:
            rec_k["kernel_trace_avg_ms"] = ms
            rec_k["valu_issue_frac"] = rec_k["SQ_INSTS_VALU"] / (ms * 1e-3) / (VALU_PEAK_GINST * 1e9)
        if "SQ_ACTIVE_INST_VALU" in rec_k:
            rec_k["active_lanes_per_valu_instruction"] = rec_k["SQ_THREAD_CYCLES_VALU"] / rec_k["SQ_ACTIVE_INST_VALU"]
        if "TCC_HIT_sum" in rec_k:
            rec_k["l2_hit_rate"] = rec_k["TCC_HIT_sum"] / (rec_k["TCC_HIT_sum"] + rec_k["TCC_MISS_sum"])
        reuse["kernels"][kname] = rec_k
    if reuse["kernels"]:
        with open(os.path.join(prof, "k_reuse_hd_sq_counters.json"), "w") as fh:
            json.dump(reuse, fh, indent=1)
        written.append("k_reuse_hd_sq_counters.json")
    # MFMA counters of the inference kernels (full-frame dispatches: the most MFMA instructions)
    lines = ["# rocprofv3 counters of the inference kernels, 1920x1080 workload (hd): one frame's candidates",
             f"# kernel sources: {sha_m} (sha256 prefix of {', '.join(KERNEL_SOURCES['mlp'])})",
             "# averages over the full-frame dispatches; counters summed over the chip"]
    have = False
    for prec, kname in (("bf16", "k_mlp_infer_bf16"), ("fp8", "k_mlp_infer_fp8")):
        c = _counters(os.path.join(outdir, f"mfma_{prec}"), kname)
        if not c.get("SQ_INSTS_MFMA"):
            continue
        have = True
        top = max(c["SQ_INSTS_MFMA"])
        sel = [i for i, v in enumerate(c["SQ_INSTS_MFMA"]) if v == top]
        avg = {k: sum(v[i] for i in sel) / len(sel) for k, v in c.items() if len(v) == len(c["SQ_INSTS_MFMA"])}
        tiles = 1920 * 1080 * 32 / 32
        lines += ["", f"## {prec.upper()} ({kname})", f"# command: {cmds['mfma_' + prec]}",
                  f"# {len(sel)} full-frame dispatches"]
        lines += [f"{k:<40s} {v:>18.0f}" for k, v in sorted(avg.items())]
        lines += ["derived:",
                  f"MFMA instructions per 32-sample tile     {avg['SQ_INSTS_MFMA'] / tiles:10.2f}",
                  f"MFMA busy cycles per MFMA instruction    {avg['SQ_VALU_MFMA_BUSY_CYCLES'] / avg['SQ_INSTS_MFMA']:10.2f}",
                  f"VALU instructions per tile (incl. MFMA)  {avg['SQ_INSTS_VALU'] / tiles:10.1f}",
                  f"MFMA cycles overlapped with VALU         "
                  f"{avg['SQ_VALU_MFMA_COEXEC_CYCLES'] / max(avg['SQ_VALU_MFMA_BUSY_CYCLES'], 1.0):10.3f}"]
    if have:
        with open(os.path.join(prof, "k_mlp_infer_hd_mfma_counters.txt"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
        written.append("k_mlp_infer_hd_mfma_counters.txt")
    return written


def time_frames(gi, torch, cfg, steps, warmup, profile_copy=False, start=0):
    """Render warm-up + timed frames of a workload with the probe target
    (frames start .. start+warmup-1, then start+warmup .. +steps-1: the
    camera pans, so the frame indices fix the views); per-pass HIP-event
    times recorded on the launch stream."""
    r = gi.Renderer(cfg, seed=1)
    r.fill_probes()
    stream = torch.cuda.current_stream()
    names = ["gbuffer", "initial", "temporal", "spatial0", "spatial1", "shade"]

    # wrap the entry points with HIP events recorded on the launch stream
    times = {k: [] for k in names}
    orig = {k: getattr(gi, k) for k in ("trace_gbuffer", "resample_initial", "resample_temporal",
                                        "resample_spatial", "shade")}
    pending = []

    def timed(key_fn, fn):
        def wrapper(*a, **kw):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn(*a, **kw)
            e1.record(stream)
            pending.append((key_fn(a), e0, e1))
        return wrapper

    gi.trace_gbuffer = timed(lambda a: "gbuffer", orig["trace_gbuffer"])
    gi.resample_initial = timed(lambda a: "initial", orig["resample_initial"])
    gi.resample_temporal = timed(lambda a: "temporal", orig["resample_temporal"])
    gi.resample_spatial = timed(lambda a: f"spatial{a[4]}", orig["resample_spatial"])
    gi.shade = timed(lambda a: "shade", orig["shade"])
    try:
        for f in range(start, start + warmup):
            r.frame(f)
        torch.cuda.synchronize()
        pending.clear()
        t0 = time.perf_counter()
        for f in range(start + warmup, start + warmup + steps):
            r.frame(f)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    finally:
        for k, v in orig.items():
            setattr(gi, k, v)
    for key, e0, e1 in pending:
        times[key].append(e0.elapsed_time(e1))
    if profile_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    W, H = r.W, r.H
    del r
    torch.cuda.empty_cache()
    return {"elapsed": elapsed, "avg": {k: (sum(v) / len(v) if v else 0.0) for k, v in times.items()},
            "W": W, "H": H}


def main():
    args = parse()
    if args.profile_commands:
        for k, v in profile_commands(os.path.abspath(args.profile_commands)).items():
            print(v)
        return
    if args.summarize_profiles:
        print("\n".join(summarize_profiles(os.path.abspath(args.summarize_profiles))))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; the path would shard by screen "
                                   "bands across GPUs, which is not implemented"}))
        sys.exit(2)
    import torch

    from paper_2108_05263_amd import build as libbuild
    if libbuild.is_stale():
        libbuild.build()
    from paper_2108_05263_amd import gi
    from paper_2108_05263_amd import scenegen as sg

    cfg = sg.CONFIGS[args.config]
    if args.mlp_ema is not None:
        MLP_OPTS["mlp_ema"] = args.mlp_ema
    if args.mlp_steps is not None:
        MLP_OPTS["mlp_steps"] = args.mlp_steps
    torch.cuda.set_device(0)
    if args.quality:
        print(json.dumps({"quality": quality(gi, sg, torch, cfg, args.quality_frames, args.quality_eval,
                                             args.ref_spp, args.quality_seeds)}), flush=True)
        return
    if args.mlp_only:
        print(json.dumps({"mlp_form": args.mlp_only,
                          **mlp_form(gi, sg, torch, cfg, args.mlp_only, args.steps, args.warmup, "always",
                                     args.mlp_train_frames)}), flush=True)
        if args.profile_copy:
            src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
        return
    if args.probe_texel != cfg.probe_texel:
        cfg = dataclasses.replace(cfg, probe_texel=args.probe_texel)
    run = time_frames(gi, torch, cfg, args.steps, args.warmup, args.profile_copy)
    elapsed, avg = run["elapsed"], run["avg"]
    W, H = run["W"], run["H"]
    npx = W * H
    ms_step = elapsed * 1e3 / args.steps
    resampling_ms = avg["initial"] + avg["temporal"] + avg["spatial0"] + avg["spatial1"] + avg["shade"]
    dom = max(avg, key=avg.get)
    dom_key = "spatial" if dom.startswith("spatial") else dom
    bytes_launch = ALGO_BYTES[dom_key] * npx
    achieved = bytes_launch / (avg[dom] * 1e-3) / 1e9
    path_bytes = sum(ALGO_BYTES[k if not k.startswith("spatial") else "spatial"] for k in avg) * npx
    line = {
        "metric": ("resampled pixels/s (1080p, M=32, 2xk=5)" if (W, H) == (1920, 1080) and cfg.glossy_frac == 0.0
                   else f"resampled pixels/s ({W}x{H}{' glossy' if cfg.glossy_frac > 0.0 else ''}, "
                        f"M={cfg.params.M}, {cfg.params.n_spatial}xk={cfg.params.k})"),
        "value": npx * args.steps / elapsed,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {W}x{H} room, {cfg.n_spheres}+{cfg.n_boxes} primitives "
                               f"({cfg.n_emitters} emitters"
                               f"{f', {cfg.glossy_frac:.0%} with a GGX layer' if cfg.glossy_frac > 0.0 else ''}), "
                               f"{cfg.probe_dims[0]}x{cfg.probe_dims[1]}x{cfg.probe_dims[2]} probes, "
                               f"M={cfg.params.M}, temporal, {cfg.params.n_spatial}x k={cfg.params.k} "
                               f"r={cfg.params.radius:g}",
                   "width": W, "height": H, "M": cfg.params.M, "k": cfg.params.k,
                   "spatial_passes": cfg.params.n_spatial, "temporal": cfg.params.temporal},
        "kernel_ms": {k: round(v, 4) for k, v in avg.items()},
        "resampling_only_pixels_per_s": npx / (resampling_ms * 1e-3),
        "path_hbm_frac": path_bytes / ((sum(avg.values())) * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {"kernel": f"k_{dom_key}", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"k_{dom_key}", cfg.name),
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "kernel_source_sha": source_sha("resampling")},
        # the dominant kernel is bound by vector-ALU issue, not HBM: its measured issue rate
        "alu_issue": alu_issue(f"k_{dom_key}", cfg.name, avg[dom]),
    }
    if dom_key == "initial" and cfg.glossy_frac == 0.0:
        # probe records the initial pass's queries read: 8 probes x (irradiance + depth
        # quad: 48 + 32 B in FP32, 24 + 16 B in binary16) per query, one query per candidate
        # (with a glossy layer the count depends on how many candidates land on glossy
        # surfaces, so it is not reported)
        qb = 8 * PROBE_RECORD_BYTES[cfg.probe_texel] * cfg.params.M * npx
        line["gather"] = {"kernel": "k_initial", "bytes_per_launch": qb, "unit": "GB/s",
                          "achieved": qb / (avg[dom] * 1e-3) / 1e9,
                          "note": "probe-record bytes read by the queries, served by L1, L2 and MALL"}
    line["config"]["probe_texel"] = cfg.probe_texel
    if cfg.probe_texel == "f32" and not args.no_f16_form:
        # the same frames from binary16 probe textures (a storage-precision option)
        h = time_frames(gi, torch, dataclasses.replace(cfg, probe_texel="f16"), args.steps, args.warmup)
        h_ms = h["elapsed"] * 1e3 / args.steps
        line["probe_f16_form"] = {"ms_per_step": h_ms, "pixels_per_s": npx * args.steps / h["elapsed"],
                                  "kernel_ms": {k: round(v, 4) for k, v in h["avg"].items()},
                                  "speed_ratio_vs_f32": ms_step / h_ms,
                                  "note": "probe texels stored as IEEE binary16 (depth as mean and variance)"}
    if not args.no_mlp and cfg.glossy_frac == 0.0:
        forms = {}
        # the cache forms are timed on later frames (after their training frames), and the
        # camera pans, so the probe form is timed again on those same frames for the ratio
        same = time_frames(gi, torch, cfg, args.steps, args.warmup, start=args.mlp_train_frames)
        same_ms = same["elapsed"] * 1e3 / args.steps
        for prec in ("bf16", "fp8"):
            for mode in ("always", "auto"):
                f = mlp_form(gi, sg, torch, cfg, prec, args.steps, args.warmup, mode, args.mlp_train_frames)
                f["probe_ms_same_frames"] = same_ms
                f["speed_ratio_vs_probe"] = same_ms / f["ms_per_step"]
                f["speed_ratio_vs_headline_frames"] = ms_step / f["ms_per_step"]
                forms[f"{prec}_{mode}"] = f
                torch.cuda.empty_cache()
        line["mlp_forms"] = forms
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, tuple(args.cpu_crop))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
