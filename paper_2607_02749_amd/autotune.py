"""Autotuner for the batched path.

The batch has four launch choices (``gv_batch_tuning`` in the C ABI): how
many workgroups the persistent kernel keeps resident per compute unit, the
order in which its atomic queue hands out instances (largest first, or input
order), and two size-class splits: the instance size up to which instances
keep their state and adjoint in one workgroup's LDS (their own persistent
kernel, one workgroup per compute unit), and the size from which instances
leave the persistent kernel and run as whole-GPU tile passes on side
streams.  (The tile shape itself, 12 tile qubits with 16 amplitudes per
lane, is fixed per prepared Hamiltonian: its off-diagonal cover and term
encoding are built for it.)  ``tune_batch``
times every candidate on the real batch with HIP events on the launching
stream and keeps the fastest; the result is cached in
a JSON file keyed by GPU architecture, precision and the batch's size class,
so later batches of the same shape skip the sweep.

The cache lives at ``$GV_TUNE_CACHE`` if set, else
``~/.cache/paper_2607_02749_amd/batch_tune.json``.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

ORDERS = {"largest_first": 0, "input": 1}
DEFAULT_BLOCKS = (1, 2, 4, 8)
DEFAULT_SPLITS = (15, 16, 17, 18, 31)   # 31: never split
DEFAULT_LDS = (-1, 12)                    # -1: no LDS-resident class


def cache_path() -> str:
    p = os.environ.get("GV_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2607_02749_amd", "batch_tune.json")


def size_class(ns: Sequence[int], layers: Sequence[int]) -> str:
    """Key of a batch's shape: qubit range, layer range and the instance
    count and total amplitude work rounded to powers of two."""
    if not ns:
        raise ValueError("empty batch")
    work = sum((1 << n) * l for n, l in zip(ns, layers))
    return (f"n{min(ns)}-{max(ns)}_L{min(layers)}-{max(layers)}"
            f"_c{1 << max(0, math.ceil(math.log2(len(ns))))}_w{math.ceil(math.log2(max(work, 1)))}")


def cache_key(arch: str, precision: str, ns: Sequence[int], layers: Sequence[int]) -> str:
    return f"{arch}/{precision}/batch/{size_class(ns, layers)}"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(key: str, entry: dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    d = load_cache(path)
    d[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def sweep(candidates: Iterable[Tuple[int, int, int, int]],
          time_ms: Callable[[int, int, int, int], float]) -> dict:
    """Time every (blocks_per_cu, order, split_n, lds_n) candidate with
    ``time_ms`` and return the fastest together with all timings."""
    timings: List[dict] = []
    for bpc, order, split, lds in candidates:
        ms = float(time_ms(bpc, order, split, lds))
        timings.append({"blocks_per_cu": bpc, "order": order, "split_n": split, "lds_n": lds,
                        "ms": ms})
    if not timings:
        raise ValueError("no candidates")
    best = min(timings, key=lambda t: t["ms"])
    return {"blocks_per_cu": best["blocks_per_cu"], "order": best["order"],
            "split_n": best["split_n"], "lds_n": best["lds_n"], "ms": best["ms"],
            "timings": timings}


def _arch(device) -> str:
    import torch
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def tune_batch(items, precision: str = "c64", blocks: Sequence[int] = DEFAULT_BLOCKS,
               orders: Sequence[int] = (0, 1), reps: int = 3, graph: bool = True,
               use_cache: bool = True, path: Optional[str] = None, device="cuda",
               splits: Sequence[int] = DEFAULT_SPLITS, lds: Sequence[int] = DEFAULT_LDS) -> dict:
    """Best launch choice for this batch (from the cache when it holds the
    batch's size class, else by timing every candidate)."""
    import torch
    from . import gv

    dev = torch.device(device)
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    ns = [an.n for an, _, _, _ in items]
    ls = [an.layers + an.final_rotation for an, _, _, _ in items]
    key = cache_key(_arch(dev), precision, ns, ls)
    if use_cache:
        hit = load_cache(path).get(key)
        if (hit and hit.get("blocks_per_cu") in blocks and hit.get("order") in orders
                and hit.get("split_n") in splits and hit.get("lds_n") in lds):
            return dict(hit, key=key, cached=True)

    def time_ms(bpc: int, order: int, split: int, lds_n: int) -> float:
        b = gv.Batch(items, precision, blocks_per_cu=bpc, order=order, graph=graph, device=dev,
                     split_n=split, lds_n=lds_n)
        b.run()                                  # warm-up (first launch loads the code object)
        torch.cuda.synchronize(dev)
        best = float("inf")
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            b.run()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        del b
        return best

    res = sweep([(bpc, o, sp, ld) for ld in lds for sp in splits for bpc in blocks for o in orders],
                time_ms)
    res["key"] = key
    res["cached"] = False
    if use_cache:
        store_cache(key, {k: res[k] for k in ("blocks_per_cu", "order", "split_n", "lds_n", "ms",
                                              "timings")}, path)
    return res


def tuned_batch(items, precision: str = "c64", graph: bool = True, device="cuda", **kw):
    """A ``gv.Batch`` built with the tuned (or cached) launch choice."""
    from . import gv
    t = tune_batch(items, precision, graph=graph, device=device, **kw)
    return gv.Batch(items, precision, blocks_per_cu=t["blocks_per_cu"], order=t["order"],
                    graph=graph, device=device, split_n=t["split_n"], lds_n=t["lds_n"])
