"""Throughput benchmark of the MLS-MPM substep on one MI355X.

A step is one substep of every particle (P2G, grid operation, G2P, F update),
with its share of the counting sort by cell: the timed window opens with a
sort and sorts every `sort_every` substeps after that, so K substeps carry
ceil(K / sort_every) sorts (when K is below the tuned interval, the interval
is set to K, which keeps exactly one sort per interval in the window).
Default workload: the 30K-particle tissue slab on a 64^3 grid pushed by a
capsule tool (dt 5e-5, E 1e4, nu 0.35), the configuration the headline
particle-substeps/s is quoted on.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config slab|large|cube|batched]

Launch options (workgroup size, particles per work item, sort interval,
graph replay, persistent kernel) come from the autotuner (which answers the
benchmark workloads from the table measured on MI355X that ships with the
package) unless --no-autotune is given; explicit flags override them.

Timing: W untimed substeps, then K substeps bracketed by device syncs and
hipEvents on the stream the library launches on.  A second pass of the same
length with the library's event timer on gives each kernel's average launch
duration; the dominant kernel's roofline uses that duration.  With the slab
workload the default run also measures the other forms: the 1M-particle slab
(`large`, with its own roofline), the 256-environment batch (eager, graph
and persistent launches), forward + adjoint, a rendered frame and other tool
shapes.  The CPU baseline is the FP64 oracle, built -O3 -march=native on
this host, threaded (per-thread node slabs, the serial result bit for bit)
on the host cores this process may use, and serial, on bounded samples of
the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3

# Algorithmic bytes (FP32 state that must cross HBM per substep):
#   per particle: read + write x (12 B) and F (36 B) = 96 B
#   per active grid node: P2G writes (m, mv) 16 B, the grid operation reads
#   them (16 B) and writes v (12 B), G2P reads v (12 B) = 56 B
# The fused G2P+P2G kernel alone moves 96 B per particle + 28 B per active node.
# With the grid operation at tile staging (one launch per substep) v never
# reaches memory: P2G writes (m, mv) 16 B and the next launch reads them 16 B,
# 32 B per active node for the substep and for its one kernel.
BYTES_PER_PARTICLE = 96
BYTES_PER_NODE_SUBSTEP = 56
BYTES_PER_NODE_FUSED = 28
BYTES_PER_NODE_GRID = 28
BYTES_PER_NODE_GAS = 32
# Forward with tape + adjoint, per particle-substep: the recorded forward (96),
# its recompute in reverse (96), the reverse substep (primal x, v, C, F read
# 96 B + adjoint x, v, C, F read and written 192 B + node adjoints ~100 B =
# ~390) and the checkpoints (96 B every 20 substeps); grid terms left out.
BYTES_PER_PARTICLE_FWD_ADJ = 96 + 96 + 390 + 96 / 20


def active_nodes(x: np.ndarray, n: int) -> int:
    """Distinct grid nodes inside the 3x3x3 stencils of the particles."""
    base = np.floor(x.astype(np.float64) * n - 0.5).astype(np.int64)
    o = np.array([(a, b, c) for a in range(3) for b in range(3) for c in range(3)])
    nodes = (base[:, None, :] + o[None, :, :]).reshape(-1, 3)
    key = (nodes[:, 0] * n + nodes[:, 1]) * n + nodes[:, 2]
    return int(np.unique(key).size)


def make_scene(name: str):
    from paper_2402_01181_amd import scenes
    if name == "slab":
        return scenes.slab_scene(), "tissue slab 30,000 particles, 64^3 grid, capsule push 0.2 m/s, slip, 1,000 substeps"
    if name == "large":
        return scenes.large_slab_scene(), "large slab 1,048,576 particles, 128^3 grid, sticky capsule pull, 500 substeps"
    if name == "cube":
        return scenes.cube_scene(), "cube 8,192 particles, 32^3 grid, no tool, 50 substeps"
    if name == "batched":
        return scenes.batched_scene(), "256 environments, 5K-50K particles each, 32^3/64^3 grids, 200 substeps"
    raise SystemExit(f"unknown config {name}")


def _events_ms(torch, fn):
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    fn()
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def measure_forms(torch, L, Sim, opts, tune, batched_steps=64, adj_steps=200, tool_steps=200, frames=40,
                  only=None):
    """The other forms of the substep on the same GPU: the 1M-particle slab,
    the batched workload (256 environments, launch options tuned for it when
    `tune`) and the
    differentiable slab (forward with tape + hand adjoint, checkpoints every
    20) against its plain forward with the slab's options, a rendered frame
    (25 substeps + the surface mesh into pinned host memory), and the slab
    with box-gripper and sampled-SDF tools in place of the capsule.  `only`
    names one of them to run alone."""
    from paper_2402_01181_amd import scenes
    out = {}
    want = lambda name: only is None or only == name
    if want("large"):
        _form_large(torch, L, Sim, tune, out)
    if want("batched"):
        _form_batched(torch, L, Sim, opts, tune, batched_steps, out)
    if want("forward_adjoint"):
        _form_forward_adjoint(torch, L, Sim, opts, adj_steps, out)
    if want("frame"):
        _form_frame(torch, L, Sim, opts, frames, out)
    if want("tool_shapes"):
        _form_tool_shapes(torch, L, Sim, opts, tool_steps, out)
    return out


def _form_batched(torch, L, Sim, opts, tune, batched_steps, out):
    """The 256-environment batch with the launch forms of the batched row:
    per-phase launches (eager), the same captured in a hipGraph, and the
    persistent kernel (a run of sort_every substeps per launch, a barrier per
    environment group), launched directly or replayed from a graph.  Each
    window opens with a sort; the form's value is the fastest variant."""
    from paper_2402_01181_amd import scenes
    bsc = scenes.batched_scene()
    bopts = dict(opts)
    if tune:
        from paper_2402_01181_amd.autotune import autotune
        bopts.update(autotune(bsc))
    se = window_sort_every(bopts.get(L.OPT_SORT_EVERY, L.OPT_DEFAULTS[L.OPT_SORT_EVERY]), batched_steps)
    bs = Sim(bsc, options={**bopts, L.OPT_GRAPH: 0, L.OPT_PERSISTENT: 0})
    nb = bsc.n_particles
    variants = {}
    for name, graph, pers in (("eager", 0, 0), ("graph", 1, 0), ("persistent", 0, 1), ("persistent_graph", 1, 1)):
        bs.set_option(L.OPT_GRAPH, graph)
        bs.set_option(L.OPT_PERSISTENT, pers)
        bs.set_option(L.OPT_SORT_EVERY, se)
        bs.step(batched_steps)        # warm-up (captures the graph)
        ms = timed_substeps(torch, L, bs, batched_steps, 0, se)
        variants[name] = {"graph": graph, "persistent": pers, "ms_per_substep": ms / batched_steps,
                          "value": nb * batched_steps / (ms * 1e-3)}
    bs.set_option(L.OPT_GRAPH, 0)
    bs.set_option(L.OPT_PERSISTENT, 0)
    x = [bs.read(L.F_X, e, device=False).T for e in range(bs.n_envs)]
    nodes = sum(active_nodes(xx, int(bs.gn[e])) for e, xx in enumerate(x))
    bytes_step = nb * BYTES_PER_PARTICLE + nodes * BYTES_PER_NODE_SUBSTEP
    best = max(variants, key=lambda k: variants[k]["value"])
    ms_sub = variants[best]["ms_per_substep"]
    out["batched"] = {"workload": "256 environments, 5K-50K particles each (seeded), 32^3/64^3 grids, own capsules",
                      "particles": nb, "substeps": batched_steps, "sort_every": se,
                      "sorts_in_window": 1 + (batched_steps - 1) // se, "used": best,
                      "graph": variants[best]["graph"], "persistent": variants[best]["persistent"],
                      "ms_per_substep": ms_sub, "value": variants[best]["value"], "unit": "particle-substeps/s",
                      "algorithmic_GBps": bytes_step / (ms_sub * 1e-3) / 1e9,
                      "hbm_frac": bytes_step / (ms_sub * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "variants": variants,
                      "options": {str(k): v for k, v in bopts.items()},
                      "status": int(any(bs.read(L.F_STATUS, e) for e in range(bs.n_envs)))}
    bs.close()
    del bs


def _form_forward_adjoint(torch, L, Sim, opts, adj_steps, out):
    from paper_2402_01181_amd import scenes
    dsc = scenes.diff_scene(substeps=adj_steps)
    ck = dsc.extra["checkpoint_every"]
    fw = Sim(dsc, options=opts)
    fw.step(20)
    ms_f = _events_ms(torch, lambda: fw.step(adj_steps))
    fw.close()
    ad = Sim(dsc, max_tape=adj_steps, checkpoint_every=ck, options=opts)
    N = dsc.n_particles
    seed = torch.full((3, N), 1.0 / N, device="cuda")
    def fwd_adj():
        ad.step(adj_steps, record_tape=True)
        ad.adjoint(adj_steps, xbar=seed)
    fwd_adj()
    ms_fa = _events_ms(torch, fwd_adj)
    gbps = N * BYTES_PER_PARTICLE_FWD_ADJ * adj_steps / (ms_fa * 1e-3) / 1e9
    ad.close()
    # the same recording kept whole in HBM (every segment's tape): the forward runs the
    # recompute passes and the adjoint only reverses
    hd = Sim(dsc, max_tape=adj_steps, checkpoint_every=ck, options=opts, hold_tape=True)
    def fwd_adj_held():
        hd.step(adj_steps, record_tape=True)
        hd.adjoint(adj_steps, xbar=seed)
    fwd_adj_held()
    ms_fh = _events_ms(torch, fwd_adj_held)
    held = {"ms_forward_with_tape_plus_adjoint": ms_fh, "ratio_to_forward": ms_fh / ms_f,
            "value": N * adj_steps / (ms_fh * 1e-3), "workspace_bytes": hd.workspace_bytes}
    hd.close()
    out["forward_adjoint"] = {"workload": f"slab 30,000 particles, 64^3, {adj_steps} substeps, checkpoints every {ck}",
                              "substeps": adj_steps, "ms_forward": ms_f, "ms_forward_with_tape_plus_adjoint": ms_fa,
                              "value": N * adj_steps / (ms_fa * 1e-3), "unit": "particle-substeps/s",
                              "ratio_to_forward": ms_fa / ms_f, "algorithmic_GBps": gbps,
                              "hbm_frac": gbps / HBM_PEAK_GBS, "held_tape": held}


def _form_tool_shapes(torch, L, Sim, opts, tool_steps, out):
    from paper_2402_01181_amd import scenes
    # the other tool shapes on the headline slab: box gripper jaws and a
    # 256^3 sampled SDF (nearest sample and trilinear), grid kernel timed
    # with the library's event timer
    tools = {}
    for name, kind, interp in (("box_gripper", "gripper", scenes.SDF_TRILINEAR),
                               ("sdf256_nearest", "sdf", scenes.SDF_NEAREST),
                               ("sdf256_trilinear", "sdf", scenes.SDF_TRILINEAR)):
        tsc = scenes.slab_tool_scene(kind, interp=interp)
        ts = Sim(tsc, options=opts)
        ts.step(20)
        ms_t = _events_ms(torch, lambda: ts.step(tool_steps))
        ts.profile(True)
        ts.step(tool_steps)
        torch.cuda.synchronize()
        ts.profile(False)
        rep = ts.profile_report()
        grid = {k: 1e3 * t / n for k, (t, n) in rep.items() if k.startswith("grid")}
        tools[name] = {"ms_per_substep": ms_t / tool_steps, "value": tsc.n_particles * tool_steps / (ms_t * 1e-3),
                       "grid_kernel_avg_us": grid, "status": int(ts.read(L.F_STATUS))}
        ts.close()
    out["tool_shapes"] = {"workload": "slab 30,000 particles, 64^3, capsule replaced by the named tool",
                          "substeps": tool_steps, "unit": "particle-substeps/s", "shapes": tools,
                          "value": min(v["value"] for v in tools.values())}


def _form_frame(torch, L, Sim, opts, frames, out):
    from paper_2402_01181_amd import scenes
    # a rendered frame as in the paper: 25 substeps, then the surface mesh
    # extracted on the device straight into pinned host memory, one sync
    import ctypes as ct
    fsc = scenes.slab_scene()
    fs = Sim(fsc, options=opts)
    fs.step(20)
    cap = 1 << 16
    host = torch.empty((cap, 3, 3), dtype=torch.float32, pin_memory=True)
    cnt = torch.zeros(1, dtype=torch.int64, pin_memory=True)
    iso = 0.5 * float(fsc.envs[0].rho)

    def extract():
        L.check(fs.lib.mpm_extract_surface(fs.ctx, 0, iso, ct.c_void_p(host.data_ptr()), cap,
                                           ct.c_void_p(cnt.data_ptr()), None), fs.ctx)

    def frame():
        fs.step(25)
        extract()
        torch.cuda.synchronize()
        if int(cnt[0]) > cap:
            raise RuntimeError("surface larger than the frame buffer")

    for _ in range(3):
        frame()
    t0 = time.perf_counter()
    for _ in range(frames):
        frame()
    ms_frame = (time.perf_counter() - t0) * 1e3 / frames
    ms_extract = _events_ms(torch, lambda: [extract() for _ in range(frames)]) / frames
    out["frame"] = {"workload": "slab 30,000 particles, 64^3: 25 substeps + surface mesh into pinned host memory",
                    "frames": frames, "ms_per_frame": ms_frame, "fps": 1e3 / ms_frame,
                    "ms_surface_extraction": ms_extract, "triangles": int(cnt[0]),
                    "value": 1e3 / ms_frame, "unit": "frames/s", "status": int(fs.read(L.F_STATUS))}
    fs.close()


def stored_traffic(config: str, kernel: str, options) -> float | None:
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or
    None when there is none or the kernels or options differ from the ones
    the counters were taken with."""
    from paper_2402_01181_amd.build import source_hash
    path = os.path.join(ROOT, "profiles", f"traffic_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != source_hash():
        return None
    from paper_2402_01181_amd import _lib as L
    shape = (L.OPT_SCHEME, L.OPT_SORT_EVERY, L.OPT_BLOCK, L.OPT_ITEM, L.OPT_PERSISTENT, L.OPT_NODE_SLOTS,
             L.OPT_GRID_AT_STAGING)
    mine = {**L.OPT_DEFAULTS, **{int(k): int(v) for k, v in options.items()}}
    theirs = {**L.OPT_DEFAULTS, **{int(k): int(v) for k, v in t.get("options", {}).items()}}
    if any(mine[k] != theirs[k] for k in shape):
        return None
    k = t.get("kernels", {}).get(kernel)
    if k is None:
        return None
    # a persistent run's dispatch covers a variable number of substeps: its
    # bytes are stored per substep and scaled by the caller
    if "bytes_per_substep" in k:
        return {"bytes_per_substep": float(k["bytes_per_substep"])}
    return float(k["bytes_per_dispatch"])


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _usable_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(scene, substeps: int, serial_substeps: int):
    """The FP64 oracle as it stands (built -O3 -march=native here) on the
    first substeps of environment 0 of the same scene: threaded over the
    host cores this process may use (at most 16, the host share of one GPU),
    and serial on a shorter sample."""
    import tempfile
    from oracle import oracle
    lib = os.path.join(tempfile.mkdtemp(prefix="mpm_oracle_native_"), "libmpm_oracle_native.so")
    oracle.use_library(oracle.build(force=True, out=lib, native=True))
    env = scene.envs[0]
    threads = max(1, min(16, _usable_cores()))
    sim = oracle.Sim(env, scene.dt, gravity=scene.gravity, bound=scene.bound)
    t0 = time.perf_counter()
    sim.run(substeps, threads=threads)
    dt_t = time.perf_counter() - t0
    ser = oracle.Sim(env, scene.dt, gravity=scene.gravity, bound=scene.bound)
    t0 = time.perf_counter()
    ser.run(serial_substeps)
    dt_s = time.perf_counter() - t0
    model = _cpu_model()
    return {"value": env.N * substeps / dt_t, "unit": "particle-substeps/s", "cores": threads, "kind": "oracle",
            "sample": f"environment 0 ({env.N} particles, {env.n}^3 grid), first {substeps} substeps, FP64 C "
                      f"(gcc -O3 -march=native) on {threads} OpenMP threads, {dt_t:.1f} s",
            "cpu_model": model, "nproc": os.cpu_count(), "usable_cores": _usable_cores(),
            "serial": {"value": env.N * serial_substeps / dt_s, "substeps": serial_substeps, "seconds": dt_s,
                       "cores": 1}}


def uses_gas(L, options, n_envs=1) -> bool:
    """The grid operation runs at tile staging (per-substep launches, or
    persistent runs for a single environment)."""
    return bool(options.get(L.OPT_GRID_AT_STAGING, 0)) and (not options.get(L.OPT_PERSISTENT, 0) or n_envs == 1)


def _roofline(rep, N, nodes, K, traffic, gas=False):
    """Roofline of the dominant kernel (by total time) from the library's
    event timer: algorithmic bytes per launch over its average duration."""
    dom = max(rep, key=lambda k: rep[k][0])
    t_ms, n_launch = rep[dom]
    avg_s = t_ms / n_launch * 1e-3
    substeps_per_launch = 1.0
    if dom.startswith("persistent"):
        # one launch runs a whole run of substeps between sorts (with the grid at
        # staging, every substep of the call but its tail)
        per_substep = N * BYTES_PER_PARTICLE + nodes * (BYTES_PER_NODE_GAS if gas else BYTES_PER_NODE_SUBSTEP)
        substeps_per_launch = ((K - 1) if gas else K) / n_launch
        per_launch = per_substep * substeps_per_launch
    elif dom.startswith("fused"):
        per_launch = N * BYTES_PER_PARTICLE + nodes * (BYTES_PER_NODE_GAS if gas else BYTES_PER_NODE_FUSED)
    elif dom.startswith("grid"):
        per_launch = nodes * BYTES_PER_NODE_GRID
    else:
        per_launch = N * BYTES_PER_PARTICLE + nodes * BYTES_PER_NODE_SUBSTEP
    achieved = per_launch / avg_s / 1e9
    measured = traffic(dom)
    if isinstance(measured, dict):
        measured = measured["bytes_per_substep"] * substeps_per_launch
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured,
            "bytes_per_launch": per_launch, "avg_launch_us": avg_s * 1e6}


def timed_substeps(torch, L, sim, K, W, sort_every):
    """W untimed substeps, then K timed substeps that open with a sort (the
    sort schedule restarts) and sort every `sort_every` after it.  Returns
    the window's milliseconds."""
    if W:
        sim.step(W)
    sim.set_option(L.OPT_SORT_EVERY, sort_every)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(K)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def event_pass(torch, L, sim, K, sort_every):
    """The same K substeps again (opening with a sort) with the library's
    event timer on: {kernel: (total ms, launches)}."""
    sim.set_option(L.OPT_GRAPH, 0)   # the event timer brackets eager launches
    sim.set_option(L.OPT_SORT_EVERY, sort_every)
    sim.profile(True)
    sim.step(K)
    torch.cuda.synchronize()
    sim.profile(False)
    return sim.profile_report()


def window_sort_every(tuned: int, K: int) -> int:
    """The sort interval used in a window of K substeps: the tuned one, or K
    when the window is shorter (one sort per interval, as in a long run)."""
    return min(int(tuned), int(K))


def _form_large(torch, L, Sim, tune, out, steps=64, warmup=10):
    """The 1,048,576-particle slab on 128^3 (the metric's second size):
    throughput over a window that opens with a sort, and the dominant
    kernel's roofline from the event pass."""
    from paper_2402_01181_amd import scenes
    sc = scenes.large_slab_scene()
    lopts = {L.OPT_SCHEME: L.SCHEME_TILED}
    if tune:
        from paper_2402_01181_amd.autotune import autotune
        lopts.update(autotune(sc))
    se = window_sort_every(lopts.get(L.OPT_SORT_EVERY, L.OPT_DEFAULTS[L.OPT_SORT_EVERY]), steps)
    ls = Sim(sc, options=lopts)
    ms = timed_substeps(torch, L, ls, steps, warmup, se)
    N = sc.n_particles
    nodes = active_nodes(ls.read(L.F_X, 0, device=False).T, int(ls.gn[0]))
    rep = event_pass(torch, L, ls, steps, se)
    kernels = {k: {"avg_us": 1e3 * t / n, "launches": n, "total_ms": t} for k, (t, n) in rep.items()}
    roof = _roofline(rep, N, nodes, steps, lambda k: stored_traffic("large", k, ls.options), uses_gas(L, ls.options))
    out["large"] = {"workload": "large slab 1,048,576 particles, 128^3 grid, sticky capsule pull along a "
                                "4-leg path at 0.2 m/s, dt 2e-5",
                    "particles": N, "substeps": steps, "sort_every": se, "sorts_in_window": 1 + (steps - 1) // se,
                    "ms_per_substep": ms / steps, "value": N * steps / (ms * 1e-3), "unit": "particle-substeps/s",
                    "active_nodes": nodes,
                    "algorithmic_GBps": (N * BYTES_PER_PARTICLE + nodes * BYTES_PER_NODE_SUBSTEP) / (ms / steps * 1e-3) / 1e9,
                    "roofline": roof, "kernels": kernels,
                    "options": {str(k): v for k, v in ls.options.items()}, "status": int(ls.read(L.F_STATUS))}
    ls.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1024)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--config", default="slab")
    ap.add_argument("--scheme", default="tiled", choices=["tiled", "direct"])
    ap.add_argument("--sort-every", type=int, default=None)
    ap.add_argument("--block", type=int, default=None)
    ap.add_argument("--item", type=int, default=None)
    ap.add_argument("--graph", type=int, default=None)
    ap.add_argument("--persistent", type=int, default=None)
    ap.add_argument("--slots", type=int, default=None, help="node-pass particles per half-wave step (1 or 3)")
    ap.add_argument("--gas", type=int, default=None, help="grid operation at tile staging (1) or a grid kernel (0)")
    ap.add_argument("--cpu-substeps", type=int, default=None,
                    help="oracle substeps for the CPU baseline (default: about 10-20 s of CPU work)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile-pass", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (launch options: library defaults plus the flags given)")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and forward+adjoint forms")
    ap.add_argument("--only-form", default=None,
                    choices=["large", "batched", "forward_adjoint", "frame", "tool_shapes"],
                    help="run just this form (with the slab's launch options, as in the default run: the "
                         "autotuner's, or the library defaults with --no-autotune, then the flags given) and print it")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_2402_01181_amd import _lib as L
    from paper_2402_01181_amd.sim import Sim

    # the workload's launch options (for --only-form the slab's, as the default run
    # passes them to the forms): the autotuner's, then the flags given
    scene, workload = make_scene("slab" if args.only_form else args.config)
    opts = {L.OPT_SCHEME: L.SCHEME_TILED if args.scheme == "tiled" else L.SCHEME_DIRECT}
    tune = not args.no_autotune and args.scheme == "tiled"
    if tune:
        from paper_2402_01181_amd.autotune import autotune, workload_key
        opts.update(autotune(scene, verbose=False))
        print(f"# autotuned options for {workload_key(scene)}: {opts}", file=sys.stderr, flush=True)
    if args.sort_every: opts[L.OPT_SORT_EVERY] = args.sort_every
    if args.block: opts[L.OPT_BLOCK] = args.block
    if args.item: opts[L.OPT_ITEM] = args.item
    if args.graph is not None: opts[L.OPT_GRAPH] = args.graph
    if args.persistent is not None: opts[L.OPT_PERSISTENT] = args.persistent
    if args.slots is not None: opts[L.OPT_NODE_SLOTS] = args.slots
    if args.gas is not None: opts[L.OPT_GRID_AT_STAGING] = args.gas
    if args.only_form:
        forms = measure_forms(torch, L, Sim, opts, tune, only=args.only_form)
        print(json.dumps(forms), flush=True)
        return
    if args.calib_copy_mib:
        a = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.5, out=b)      # one elementwise kernel: reads and writes the stated MiB
        torch.cuda.synchronize()
        del a, b
    sim = Sim(scene, options=opts)
    N = scene.n_particles
    K, W = args.steps, args.warmup
    se = window_sort_every(sim.options.get(L.OPT_SORT_EVERY, L.OPT_DEFAULTS[L.OPT_SORT_EVERY]), K) \
        if args.scheme == "tiled" else sim.options.get(L.OPT_SORT_EVERY, L.OPT_DEFAULTS[L.OPT_SORT_EVERY])
    sorts = 1 + (K - 1) // se if args.scheme == "tiled" else 0

    print(f"# bench: {workload}; N={N}; warmup {W}, timed {K} substeps opening with a sort, sort every {se} "
          f"({sorts} sorts in the window)", file=sys.stderr, flush=True)
    ms = timed_substeps(torch, L, sim, K, W, se)
    value = N * K / (ms * 1e-3)
    print(f"# timed: {ms:.3f} ms, {value:.4g} particle-substeps/s", file=sys.stderr, flush=True)

    status = [sim.read(L.F_STATUS, e) for e in range(sim.n_envs)]
    x_final = [sim.read(L.F_X, e, device=False).T for e in range(sim.n_envs)]
    nodes = sum(active_nodes(x, int(sim.gn[e])) for e, x in enumerate(x_final))

    roofline, kernels = None, {}
    if not args.no_profile_pass:
        rep = event_pass(torch, L, sim, K, se)
        kernels = {k: {"avg_us": 1e3 * t / n, "launches": n, "total_ms": t} for k, (t, n) in rep.items()}
        roofline = _roofline(rep, N, nodes, K, lambda k: stored_traffic(args.config, k, sim.options),
                             uses_gas(L, sim.options))
        print(f"# kernels: " + ", ".join(f"{k} {v['avg_us']:.2f}us x{v['launches']}" for k, v in kernels.items()),
              file=sys.stderr, flush=True)

    forms = None
    if not args.no_forms and args.config == "slab":
        sim.close()
        forms = measure_forms(torch, L, Sim, {k: v for k, v in opts.items() if k != L.OPT_GRAPH}, tune)
        for k, v in forms.items():
            print(f"# form {k}: {v['value']:.4g} {v.get('unit', 'particle-substeps/s')}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        default_cpu = {"slab": (1000, 300), "large": (20, 10), "cube": (200, 200), "batched": (400, 200)}
        sub, ser = default_cpu.get(args.config, (50, 50))
        if args.cpu_substeps:
            sub = ser = args.cpu_substeps
        cpu = cpu_baseline(scene, sub, ser)
        print(f"# cpu baseline: {cpu['value']:.4g} particle-substeps/s on {cpu['cores']} threads "
              f"({cpu['cpu_model']}), serial {cpu['serial']['value']:.4g}", file=sys.stderr, flush=True)

    out = {
        "metric": "particle-substeps/sec",
        "value": value,
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded particles in a box, analytic capsule tool)",
        "config": {"workload": workload, "config": args.config, "particles": N,
                   "grid": [int(g) for g in sim.gn[:4]], "envs": sim.n_envs, "substeps_timed": K,
                   "sort_every": se, "sorts_in_window": sorts,
                   "scheme": args.scheme, "options": {str(k): v for k, v in sim.options.items()},
                   "active_nodes": nodes,
                   "algorithmic_bytes_per_substep": N * BYTES_PER_PARTICLE + nodes * (
                       BYTES_PER_NODE_GAS if uses_gas(L, sim.options) else BYTES_PER_NODE_SUBSTEP)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "forms": forms,
        "status": status if any(status) else 0,
    }
    print(json.dumps(out), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
