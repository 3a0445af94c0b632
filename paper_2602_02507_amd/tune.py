"""Autotuner of the contraction launches.

The two angular contractions have three launch knobs (the C ABI's
mpole_tuning): the output tile height of the moment and of the expansion
contraction (64 or 128 shells per tile for the split precisions; 64 for
FP64), and the workgroup target of the moment contraction, whose K dimension
(the blocks of a shell) is split over that many workgroups.  None of them
changes what is summed, only how the sums are tiled and split.

The tuner times candidate choices on the device with the library's own
per-phase HIP events, keeps the fastest per contraction (moment: moment +
split-K reduction time; expansion: expansion time), and caches the result in
a JSON file keyed by device, precision and the shape of the mesh (sizes,
lmax and the rows x blocks of each coarsening class), so a shape is measured
once per device.  Timing does not depend on the density values, so the
candidates are timed on a constant density.

For a batch, each field's tile heights come from tuning that field alone;
the moment targets, which matter for how the fields share the GPU, are then
chosen by timing the whole batch at a few multiples of each field's share of
one round of resident workgroups (cached per device and set of field shapes).
"""
import json
import os
import time

import numpy as np

from . import mpole

CACHE_ENV = "MPOLE_TUNE_CACHE"


def cache_path():
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "mpole", "tune.json")


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data, path=None):
    path = path or cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # an unwritable cache only costs re-tuning


def class_shape(mesh):
    """(rows, blocks) of each coarsening class with at least one shell."""
    if mesh.shell_class is None:
        return [(int(mesh.nr), int(mesh.ntheta * mesh.nphi))]
    sc = np.asarray(mesh.shell_class)
    cb = np.asarray(mesh.class_block).reshape(-1, mesh.ntheta * mesh.nphi)
    return [(int((sc == c).sum()), int(cb[c].max()) + 1) for c in range(cb.shape[0]) if (sc == c).any()]


def shape_key(mesh, precision, device_name):
    cls = ";".join("%dx%d" % rb for rb in class_shape(mesh))
    return "%s|%s|%dx%dx%d|L%d|%s" % (device_name, precision, mesh.nr, mesh.ntheta, mesh.nphi, mesh.lmax, cls)


def _device_name(device):
    """Architecture and compute-unit count of the device (stable key part)."""
    import torch
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "") or p.name
    return ("%s/%dcu" % (arch.split(":")[0], p.multi_processor_count)).replace("|", "/")


def candidates(precision):
    """(moment candidates, expansion candidates) as partial tunings."""
    if precision in ("fp64sep", "bf16x3sep"):   # the separable paths have no launch knobs
        mom, exp = [{"moment_wgs": 0}], [{"expand_tile_m": 0}]
    elif precision == "fp64":
        mom = [{"moment_wgs": w, "moment_tile_m": 64} for w in (512, 1024, 2048, 4096)]
        exp = [{"expand_tile_m": 64}]
    else:
        mom = [{"moment_wgs": w, "moment_tile_m": h} for h in (128, 64) for w in (384, 768, 1536, 3072)]
        exp = [{"expand_tile_m": h} for h in (128, 64)]
    return mom, exp


def _time_plan(mesh, precision, device, rho, tuning, warmup, reps):
    plan = mpole.Plan.from_mesh(mesh, precision=precision, device=device, tuning=tuning)
    out = plan.empty_outputs(ang=False, interior=False, exterior=False)
    for _ in range(warmup):
        plan.solve_into(rho, **out)
    plan.set_timing(True)
    plan.phase_ms()
    for _ in range(reps):
        plan.solve_into(rho, **out)
    ph = plan.phase_ms()
    plan.set_timing(False)
    per = {k: v[0] / max(v[1], 1) for k, v in ph.items()}
    return per


def tune_plan(mesh, precision="bf16x3", device="cuda", warmup=1, reps=3, cache=None, log=None):
    """Fastest tuning (dict of the three knobs) for one mesh, from the cache
    when the shape was tuned before on this device.  `cache` is a dict that
    is read and updated in place (saved by the caller); None uses the file."""
    import torch
    dev = torch.device(device)
    if dev.index is None:
        dev = torch.device(dev.type, torch.cuda.current_device())
    own = cache is None
    if own:
        cache = load_cache()
    key = shape_key(mesh, precision, _device_name(dev))
    hit = cache.get(key)
    if hit is not None:
        return dict(hit["tuning"])
    rho = torch.ones((mesh.nr, mesh.ntheta, mesh.nphi), dtype=torch.float64, device=dev)
    mom_c, exp_c = candidates(precision)
    t0 = time.perf_counter()
    best_m, best_m_ms, best_e, best_e_ms = None, float("inf"), None, float("inf")
    trials = []
    for c in mom_c:
        per = _time_plan(mesh, precision, dev, rho, c, warmup, reps)
        ms = per["moment"] + per["reduce"]
        trials.append(("moment", c, ms))
        if ms < best_m_ms:
            best_m, best_m_ms = c, ms
    for c in exp_c:
        per = _time_plan(mesh, precision, dev, rho, c, warmup, reps)
        ms = per["expand"]
        trials.append(("expand", c, ms))
        if ms < best_e_ms:
            best_e, best_e_ms = c, ms
    del rho
    tuning = {"moment_wgs": best_m.get("moment_wgs", 0), "moment_tile_m": best_m.get("moment_tile_m", 0),
              "expand_tile_m": best_e.get("expand_tile_m", 0)}
    cache[key] = {"tuning": tuning, "moment_ms": best_m_ms, "expand_ms": best_e_ms,
                  "seconds": time.perf_counter() - t0}
    if log:
        log("tune %s -> %s (moment+reduce %.4f ms, expand %.4f ms; %d trials)"
            % (key, tuning, best_m_ms, best_e_ms, len(trials)))
    if own:
        save_cache(cache)
    return tuning


def _time_batch(meshes, precision, rho, device, tunings, warmup, reps):
    import torch
    b = mpole.Batch(meshes, precision=precision, rho=rho, device=device, tunings=tunings)
    for _ in range(warmup):
        b.solve()
    torch.cuda.synchronize(device)
    s = torch.cuda.current_stream(device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        b.solve()
    e1.record(s)
    torch.cuda.synchronize(device)
    del b
    return e0.elapsed_time(e1) / reps


def tune_batch(meshes, precision="bf16x3", device="cuda", rho=None, warmup=1, reps=3, log=None):
    """Per-field tunings for a batch: tile heights tuned per field shape
    (cached), moment targets chosen by timing the whole batch.  Returns
    (list of per-field tuning dicts, info dict)."""
    import torch
    dev = torch.device(device)
    if dev.index is None:
        dev = torch.device(dev.type, torch.cuda.current_device())
    t0 = time.perf_counter()
    cache = load_cache()
    n_before = sum(1 for k in cache if not k.startswith("batch|"))
    tiles = [tune_plan(m, precision, dev, warmup, reps, cache=cache, log=log) for m in meshes]
    save_cache(cache)
    t_fields = time.perf_counter() - t0
    if rho is None:
        rho = [torch.ones((m.nr, m.ntheta, m.nphi), dtype=torch.float64, device=dev) for m in meshes]
    # default shares of the moment workgroups (as the library computes them)
    shares = _default_shares(meshes, precision)
    import hashlib
    bkey = "batch|%s|%s|%s" % (_device_name(dev), precision, hashlib.sha1(
        "\n".join(shape_key(m, precision, "") for m in meshes).encode()).hexdigest()[:16])
    make = lambda mult: [{"moment_wgs": max(1, int(round(mult * s))), "moment_tile_m": t["moment_tile_m"],
                          "expand_tile_m": t["expand_tile_m"]} for s, t in zip(shares, tiles)]
    trials = []
    if bkey in cache:
        best = make(cache[bkey]["mult"])
    else:
        best_mult, best_ms = None, float("inf")
        for mult in (1, 2, 4):
            ms = _time_batch(meshes, precision, rho, dev, make(mult), warmup, reps)
            trials.append((mult, ms))
            if log:
                log("tune batch: moment share x%d -> %.3f ms" % (mult, ms))
            if ms < best_ms:
                best_mult, best_ms = mult, ms
        best = make(best_mult)
        cache[bkey] = {"mult": best_mult, "batch_ms": best_ms, "trials_ms": trials}
        save_cache(cache)
    info = {"field_shapes_tuned": sum(1 for k in cache if not k.startswith("batch|")) - n_before,
            "field_shapes": len(meshes), "field_tuning_s": t_fields, "batch_trials_ms": trials,
            "seconds": time.perf_counter() - t0, "cache": cache_path()}
    return best, info


def _default_shares(meshes, precision):
    """Each field's default moment workgroup target inside a batch: its share
    of one round of resident workgroups, in proportion to its moment work."""
    work = []
    for m in meshes:
        namp = -(-(m.lmax + 1) ** 2 // 16) * 16
        w = 0.0
        for rows, blocks in class_shape(m):
            w += rows * (-(-blocks // 16) * 16) * namp
        work.append(w)
    total = max(sum(work), 1.0)
    rnd = 1024 if precision == "fp64" else 768
    return [max(1.0, rnd * w / total) for w in work]
