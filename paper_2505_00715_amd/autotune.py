"""Autotuner of the library's launch parameters (``gcq_tuning``) for one workload.

The search times the library's own calls on the caller's operator, with the
HIP-event device times the library records (``Context.kernel_ms``):

  aca_waves            wave64s per (block, frequency) pair of ``aca_blocks``: 1, 2, 4
  aca3d_waves          wave64s per admissible block of ``aca3d``, per size class
  aca3d_stack_slices   initial stack reservation of an admissible block: 4, 8, 16
  product_graph        per-frequency product as a replayed graph or plain launches
  product_cols_per_wave  frequency columns per wave64 of the split-bf16 product: 32, 64

Results are cached as JSON, keyed by (workload key, device architecture,
precision).  Every candidate is a valid configuration: results differ only in
rounding order, never in what is computed.
"""
from __future__ import annotations

import json
import os
import time

from . import C64, C64_SPLIT_BF16, FLAG_RECOMPRESS, PER_FREQUENCY

ACA3D_CANDIDATES = [(4, 4, 4, 4), (2, 4, 4, 4), (2, 2, 4, 4), (4, 4, 4, 8), (1, 2, 4, 8)]
STACK_CANDIDATES = [4, 8, 16]


def choose_product_graph(times: dict) -> int:
    """Graph replay (1) or plain launches (0) from the product's times under
    each.  The graph setting also runs the solver's Arnoldi step on the device,
    which leaves converged frequency tiles out of the product (a gain the single
    product does not show), so plain launches win only when clearly faster."""
    return 0 if times[0] < 0.97 * times[1] else 1


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "gcqbem", "tuning.json")


def device_arch(device: int = 0) -> str:
    import torch
    p = torch.cuda.get_device_properties(device)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _key(workload: str, arch: str, precision: int) -> str:
    return f"{workload}|{arch}|{'c64' if precision == C64 else 'c128'}"


def load(workload: str, precision: int, path: str | None = None, device: int = 0):
    path = path or default_cache_path()
    try:
        with open(path) as fh:
            return json.load(fh).get(_key(workload, device_arch(device), precision))
    except (OSError, ValueError):
        return None


def save(workload: str, precision: int, params: dict, path: str | None = None, device: int = 0):
    path = path or default_cache_path()
    data = {}
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        data = {}
    data[_key(workload, device_arch(device), precision)] = params
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # a read-only cache location only costs a re-tune


def apply(ctx, params: dict):
    ctx.set_tuning(aca3d_waves=params["aca3d_waves"], aca3d_stack_slices=params["aca3d_stack_slices"],
                   aca_waves=params["aca_waves"], product_graph=params["product_graph"],
                   product_cols_per_wave=params.get("product_cols_per_wave", 32))


def tune(ctx, workload: str, precision: int, tol: float, max_rank: int = 64, max_freq_rank: int = 40,
         aca_flags: int = FLAG_RECOMPRESS, X=None, Y=None, path: str | None = None,
         use_cache: bool = True, log=None, aca_freq_idx=None, aca3d_candidates=None,
         stack_candidates=None, product_precision: int | None = None) -> dict:
    """Search the launch parameters on ``ctx`` (mesh, frequencies and tree set
    up) and leave the best ones set.  X, Y: device buffers for the product
    (optional).  aca_freq_idx: representatives the aca_blocks candidates are
    timed on (None: all; a subset keeps the search affordable on large
    workloads); aca3d_candidates, stack_candidates: the group-size sets and
    stack reservations to try (a large reservation on a large workload may not
    fit the device);
    product_precision: precision of the product timed (default: precision).
    Returns the chosen parameters with their measured times."""
    if use_cache:
        cached = load(workload, precision, path)
        if cached is not None:
            apply(ctx, cached)
            return dict(cached, source="cache")
    say = log or (lambda *_: None)
    t0 = time.perf_counter()
    best = {}
    # waves per pair of the per-frequency ACA
    times = {}
    for w in (1, 2, 4):
        ctx.set_tuning(aca_waves=w)
        ctx.aca_blocks(tol, max_rank, precision, aca_flags, freq_idx=aca_freq_idx)
        times[w] = ctx.kernel_ms("aca_total")
        say(f"[autotune] aca_waves {w}: {times[w]:.1f} ms")
    best["aca_waves"] = min(times, key=times.get)
    ctx.set_tuning(aca_waves=best["aca_waves"])
    # 3D-ACA group sizes, then the stack reservation
    times = {}
    for c in (aca3d_candidates or ACA3D_CANDIDATES):
        ctx.set_tuning(aca3d_waves=c, aca3d_stack_slices=8)
        st = ctx.aca3d(tol, tol, max_freq_rank, precision)
        times[c] = st.far_ms
        say(f"[autotune] aca3d_waves {c}: {times[c]:.1f} ms")
    best["aca3d_waves"] = list(min(times, key=times.get))
    times = {}
    for sl in (stack_candidates or STACK_CANDIDATES):
        ctx.set_tuning(aca3d_waves=best["aca3d_waves"], aca3d_stack_slices=sl)
        st = ctx.aca3d(tol, tol, max_freq_rank, precision)
        times[sl] = st.far_ms
        say(f"[autotune] aca3d_stack_slices {sl}: {times[sl]:.1f} ms")
    best["aca3d_stack_slices"] = min(times, key=times.get)
    ctx.set_tuning(aca3d_stack_slices=best["aca3d_stack_slices"])
    best["aca3d_ms"] = times[best["aca3d_stack_slices"]]
    ctx.aca3d(tol, tol, max_freq_rank, precision)   # the operator of the chosen setting
    # the product: graph replay or plain launches, then (split-bf16) the
    # frequency columns per wave
    best["product_graph"] = 1
    best["product_cols_per_wave"] = 32
    if X is not None and Y is not None:
        import torch
        pprec = product_precision if product_precision is not None else precision

        def product_ms():
            ts = []
            for _ in range(4):
                ctx.compressed_matvec(PER_FREQUENCY, pprec, X, Y)
                torch.cuda.synchronize()
                ts.append(ctx.kernel_ms("matvec_perfreq"))
            return sorted(ts)[len(ts) // 2]
        times = {}
        for gr in (0, 1):
            ctx.set_tuning(product_graph=gr)
            times[gr] = product_ms()
            say(f"[autotune] product_graph {gr}: {times[gr]:.3f} ms")
        best["product_graph"] = choose_product_graph(times)
        ctx.set_tuning(product_graph=best["product_graph"])
        if pprec == C64_SPLIT_BF16:
            times = {}
            for cw in (32, 64):
                ctx.set_tuning(product_cols_per_wave=cw)
                times[cw] = product_ms()
                say(f"[autotune] product_cols_per_wave {cw}: {times[cw]:.3f} ms")
            best["product_cols_per_wave"] = min(times, key=times.get)
    apply(ctx, best)
    best["tuning_s"] = time.perf_counter() - t0
    save(workload, precision, best, path)
    return dict(best, source="search")
