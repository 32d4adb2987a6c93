"""Launch-shape autotuner for the fused sweep.

For a lattice shape, storage type and mask kind (none; walls that fill
whole rows; any other mask) it times the fused sweep
over a grid of launch shapes (rows a wavefront marches, wavefronts per
workgroup, XCD remap on/off, one or two columns per lane where two apply,
one, two or three time steps per launch where they apply) on a scratch lattice of
that shape, and keeps the fastest.  For a batch it times the batched step (rows, wavefronts per
workgroup, XCD remap) on scratch copies of the members.  Results persist in
a JSON cache keyed by GPU architecture, storage, mask kind and size
buckets (for a batch: its member count and size mix); the cache path is
$TRTLBM_TUNE_CACHE, else ~/.cache/trtlbm/tune.json.
"""
from __future__ import annotations

import json
import math
import os
import time

ROWS = (4, 8, 16, 32, 64, 128)
WAVES = (1, 2, 4)            # one column per lane: at most 4 wavefronts per workgroup
WAVES_PAIR = (1, 2, 4, 8, 16)  # two columns per lane (the library caps FP64 at 8)
REMAP = (1, 0)
COLS = (1, 2)
TB2_ROWS = (8, 12, 16, 20, 24, 30, 32, 37, 48, 64)  # two time steps per launch
TB2_WAVES = (1, 2, 4)
TB2_PREFETCH = (1, 2)  # rows ahead of their use that the two-step loads run
TB3_ROWS = (8, 12, 16, 20, 24, 32, 38, 40, 48, 64, 96)  # three time steps per launch (FP32)
TB2_VALID, TB3_VALID = 120, 116  # columns a wavefront stores in the two- and three-step passes
SIMDS = 1024  # 256 CUs x 4 SIMDs


def whole_round_rows(nx: int, ny: int, valid: int, waves_per_block: int,
                     resident_per_simd: int, rounds=(1, 2, 3)):
    """Rows per wavefront that make the workgroups of a multi-step pass fill
    the machine in whole rounds: for k rounds, the shortest rows whose
    workgroup count (row blocks x window groups) is at most k times the
    workgroups resident at once (SIMDs x wavefronts per SIMD / wavefronts
    per workgroup).  The measured optimum often sits at such a count (4096^2,
    three steps per launch: 74 rows, 504 workgroups of 512 resident, 87.6
    us per step against 91.0 at 48 rows)."""
    windows = (nx + valid - 1) // valid
    groups = (windows + waves_per_block - 1) // waves_per_block
    slots = SIMDS * resident_per_simd // waves_per_block
    out = set()
    for k in rounds:
        blocks = k * slots // groups
        if blocks < 1:
            continue
        r = (ny + blocks - 1) // blocks
        if 8 <= r <= 512:
            out.add(r)
    return sorted(out)


def cache_path() -> str:
    return os.environ.get("TRTLBM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "trtlbm", "tune.json"))


def _bucket(v: int) -> int:
    """Power-of-two size bucket (64, 128, ..., 32768)."""
    return 1 << max(6, min(15, int(round(math.log2(max(1, v))))))


def key(nx: int, ny: int, storage: str, has_mask: bool, arch: str = "gfx950",
        walls: bool = False) -> str:
    """Cache key: storage, the lattice's kind (open; a mask whose solid
    nodes fill whole rows, walls; any other mask or open x boundaries) and
    the size buckets."""
    kind = ("walls" if walls else "mask") if has_mask else "open"
    return "%s|%s|%s|%d|%d" % (arch, storage, kind, _bucket(nx), _bucket(ny))


def row_walls(mask, inflow=None) -> bool:
    """Whether a host mask's solid nodes fill whole rows (and x is periodic):
    such FP32 and FP16 lattices take the multi-step passes as open ones do."""
    if mask is None or inflow is not None:
        return False
    import numpy as np
    m = np.asarray(mask) != 0
    return bool(np.all(m == m[:, :1]))


def load_cache(path: str | None = None) -> dict:
    try:
        with open(path or cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str | None = None) -> bool:
    """Write the cache atomically; False (and nothing raised) where the
    cache location is not writable -- tuning results then last for the
    process only."""
    path = path or cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        return False
    return True


def candidates(nx: int, ny: int, has_mask: bool = False, storage: str = "f32",
               walls: bool = False):
    """Launch shapes (rows, waves per workgroup, XCD remap, columns per
    lane, graph sweeps (0: default), time steps per launch, prefetch rows (0:
    automatic)) worth timing.  Two columns per lane apply to every width
    that is not 1 mod 128 (with or without a mask: masked lattices use the
    link map); two time steps per launch to FP32 and FP16 lattices without a
    mask, whose loads run one or two rows ahead; three to such FP32
    lattices.  walls (with has_mask): the mask's solid nodes fill whole
    rows, so the lattice takes two and three steps as an open one does."""
    cols = COLS if nx % 128 != 1 else (1,)
    out = []
    for c in cols:
        waves = WAVES if c == 1 else tuple(w for w in WAVES_PAIR
                                            if storage != "f64" or w <= 8)
        for r in ROWS:
            if r > max(4, ny):
                continue
            for w in waves:
                for x in REMAP:
                    out.append((r, w, x, c, 0, 1, 0))
    multi = not has_mask or walls
    if storage in ("f32", "f16") and multi:
        for r in TB2_ROWS:
            if r > max(8, ny):
                continue
            for w in TB2_WAVES:
                for x in REMAP:
                    for p in TB2_PREFETCH:
                        out.append((r, w, x, 2, 0, 2, p))
        # FP32 loading two rows ahead keeps two wavefronts per SIMD, else three
        for w in TB2_WAVES:
            for p in TB2_PREFETCH:
                per = 2 if (storage == "f32" and p == 2) or storage == "f64" else 3
                for r in whole_round_rows(nx, ny, TB2_VALID, w, per):
                    if r in TB2_ROWS:
                        continue
                    for x in REMAP:
                        out.append((r, w, x, 2, 0, 2, p))
    if storage == "f32" and multi:
        for r in TB3_ROWS:
            if r > max(8, ny):
                continue
            for w in TB2_WAVES:
                for x in REMAP:
                    out.append((r, w, x, 2, 0, 3, 1))
        # two wavefronts per SIMD (238 VGPRs)
        for w in TB2_WAVES:
            for r in whole_round_rows(nx, ny, TB3_VALID, w, 2):
                if r in TB3_ROWS:
                    continue
                for x in REMAP:
                    out.append((r, w, x, 2, 0, 3, 1))
    return out


def time_shape(lat, shape, steps: int, warmup: int) -> float:
    """Milliseconds per sweep for one launch shape on lattice `lat`."""
    import torch
    lat.set_tuning(*shape)
    lat.step(warmup)
    lat.prepare(steps)   # graph capture stays out of the timed region
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    lat.step(steps)
    end.record(lat.stream)
    end.synchronize()
    return start.elapsed_time(end) / steps


def tune(nx: int, ny: int, storage: str = "f32", mask=None, steps: int | None = None,
         shapes=None, log=None) -> dict:
    """Time every candidate launch shape; returns {"best": shape, "ms": ...,
    "table": [(shape, ms), ...]}.  The scratch lattice starts at rest."""
    import numpy as np

    from .lattice import Lattice
    lat = Lattice(nx, ny, 0.6, 1.0, storage=storage, mask=mask)
    lat.init_equilibrium(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    if steps is None:
        steps = max(10, min(400, int(2e9 / max(1, nx * ny))))
    table = []
    for shape in shapes or candidates(nx, ny, mask is not None, storage, row_walls(mask)):
        ms = time_shape(lat, shape, steps, max(2, steps // 10))
        table.append((list(shape), ms))
        if log:
            log("tune %dx%d %s %s: %.4f ms" % (nx, ny, storage, shape, ms))
    lat.close()
    table.sort(key=lambda t: t[1])
    return {"best": table[0][0], "ms": table[0][1], "table": table,
            "when": time.strftime("%Y-%m-%dT%H:%M:%S")}


def best_shape(nx: int, ny: int, storage: str = "f32", has_mask: bool = False,
               autotune: bool = False, log=None, walls: bool = False):
    """Cached best launch shape, tuning (and caching) on a miss when
    `autotune` is set; None when unknown (the library default applies).
    With a mask it is tuned on a channel (walls on the first and last rows),
    plus, unless `walls`, a solid node off those rows."""
    cache = load_cache()
    k = key(nx, ny, storage, has_mask, walls=walls)
    if k in cache:
        return tuple(cache[k]["best"])
    if not autotune:
        return None
    mask = None
    if has_mask:
        import numpy as np
        mask = np.zeros((ny, nx), np.uint8)
        mask[0] = mask[-1] = 1
        if not walls and ny > 2:
            mask[ny // 2, nx // 2] = 1
    res = tune(nx, ny, storage, mask=mask, log=log)
    cache[k] = {"best": res["best"], "ms": res["ms"], "when": res["when"]}
    save_cache(cache)
    return tuple(res["best"])


# Batched launches: rows per wavefront (0: per the row policy below),
# wavefronts per workgroup (at most 4) and XCD remap; each member keeps its
# column mode.  Row policies (trt_tuning.batch_items): -1 each member's own
# automatic rows; n > 0 one batch-wide cap leaving at least n work items
# (members no taller than the cap in one item per strip).  Orders
# (batch_order): 1 member by member, 2 costliest items first.
BATCH_ROWS = (4, 8, 16, 32)
BATCH_WAVES = (2, 4)
BATCH_ITEMS = (-1, 16384, 32768)
BATCH_ORDERS = (1, 2)


def batch_candidates():
    """Launch shapes (rows, waves per workgroup, XCD remap, columns, row
    policy, order) worth timing for a batch: uniform rows, and the two row
    policies in both orders."""
    out = [(r, w, x, 0, 0, 1) for r in BATCH_ROWS for w in BATCH_WAVES for x in REMAP]
    out += [(0, w, x, 0, i, o) for i in BATCH_ITEMS for o in BATCH_ORDERS for w in BATCH_WAVES
            for x in REMAP]
    return out


def batch_key(sizes, storage: str, has_mask: bool, arch: str = "gfx950") -> str:
    """Cache key of a batch: storage, mask presence, member count and the
    members' node counts in power-of-two buckets (the shape of the work, not
    its exact sizes)."""
    hist = {}
    for nx, ny in sizes:
        b = _bucket(int(round(math.sqrt(max(1, nx * ny)))))
        hist[b] = hist.get(b, 0) + 1
    comp = ",".join("%dx%d" % (b, hist[b]) for b in sorted(hist))
    return "%s|%s|%s|batch|%d|%s" % (arch, storage, "mask" if has_mask else "open",
                                     len(sizes), comp)


def time_batch_shape(batch, shape, steps: int, warmup: int) -> float:
    """Milliseconds per batched step for one launch shape."""
    import torch
    batch.set_tuning(*shape)
    batch.step(warmup)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(batch.stream)
    batch.step(steps)
    end.record(batch.stream)
    end.synchronize()
    return start.elapsed_time(end) / steps


def tune_batch(lattices, steps: int | None = None, shapes=None, log=None) -> dict:
    """Time every candidate batch launch shape on scratch copies of the
    members (same sizes, relaxation times, forces, masks, open boundaries
    and storage, started at rest), so the batch's own state is untouched;
    returns {"best": shape, "ms": ..., "table": [(shape, ms), ...]}."""
    import numpy as np

    from .lattice import Batch, Lattice
    scratch = []
    try:
        for l in lattices:
            mask = None if l.mask is None else l.mask.cpu().numpy()
            s = Lattice(l.nx, l.ny, l.tau_s, l.tau_s2, g=l.g, mask=mask, storage=l.storage,
                        device=l.device, inflow=l.inflow)
            s.init_equilibrium(np.ones((l.ny, l.nx)), np.zeros((l.ny, l.nx)),
                               np.zeros((l.ny, l.nx)))
            scratch.append(s)
        nodes = sum(l.nx * l.ny for l in lattices)
        if steps is None:
            steps = max(10, min(200, int(4e9 / max(1, nodes))))
        b = Batch(scratch)
        table = []
        try:
            for shape in shapes or batch_candidates():
                ms = time_batch_shape(b, shape, steps, max(2, steps // 10))
                table.append((list(shape), ms))
                if log:
                    log("tune batch of %d %s: %.4f ms" % (len(lattices), shape, ms))
        finally:
            b.close()
    finally:
        for s in scratch:
            s.close()
    table.sort(key=lambda t: t[1])
    return {"best": table[0][0], "ms": table[0][1], "table": table,
            "when": time.strftime("%Y-%m-%dT%H:%M:%S")}


def best_batch_shape(lattices, autotune: bool = False, log=None):
    """Cached best launch shape of a batch of these lattices, tuning (and
    caching) on a miss when `autotune` is set; None when unknown (the
    library default applies)."""
    lats = list(lattices)
    k = batch_key([(l.nx, l.ny) for l in lats], lats[0].storage,
                  any(l.mask is not None or l.inflow is not None for l in lats))
    cache = load_cache()
    if k in cache:
        return tuple(cache[k]["best"])
    if not autotune:
        return None
    res = tune_batch(lats, log=log)
    cache[k] = {"best": res["best"], "ms": res["ms"], "when": res["when"]}
    save_cache(cache)
    return tuple(res["best"])
