"""Autotuner of the operator's launch-shaping parameters, by measurement on the device.

Tunables: the cluster-tree leaf level (it trades near-field non-zeros against coupling
blocks and so decides the matvec's bytes and the assembly's work) and the coupling kernel's
chunk width (columns of an owner's coupling rows per wave).  Each candidate is planned on
the host, skipped if its operator workspace exceeds the budget, assembled, and timed over a
number of applies with HIP events; the fastest apply wins.  Results can be cached in a JSON
file keyed by the workload's shape.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import BEM_PREC_FP64, Operator


def _time_apply(op: Operator, nrhs: int, steps: int) -> float:
    dt = op.space.dtype
    x = torch.randn((nrhs, op.ndof), dtype=torch.float64, device="cuda")
    if dt == torch.complex128:
        x = torch.complex(x, torch.randn_like(x))
    y = torch.empty_like(x)
    for _ in range(3):
        op.apply(x, out=y)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        op.apply(x, out=y)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps * 1e3  # microseconds


def tune(space, q: int = 5, eta: float = 1.6, nrhs: int = 1, leaf_levels=None, chunks=(128, 256, 512),
         steps: int = 20, budget_bytes: float = 16e9, cache: str | None = None) -> dict:
    """Returns {"leaf_level", "chunk_cols", "apply_us", "table": [...]} for the space."""
    L = space.level
    key = f"g{space.geom.kind}_L{L}_d{space.degree}_k{space.kernel}_q{q}_eta{eta}_r{nrhs}"
    if cache and os.path.exists(cache):
        with open(cache) as f:
            got = json.load(f).get(key)
        if got:
            return got
    if leaf_levels is None:
        leaf_levels = [lv for lv in range(max(L - 3, 0), L + 1)]
    batch = nrhs if nrhs > 1 else 0
    table = []
    best = None
    for leaf in leaf_levels:
        op = Operator(space, q=q, eta=eta, leaf_level=leaf, assemble=False, batch_rhs=batch)
        if op.info.op_bytes > budget_bytes:
            table.append({"leaf_level": leaf, "chunk_cols": 0, "skipped": f"{op.info.op_bytes/1e9:.1f} GB"})
            continue
        t0 = time.perf_counter()
        op.assemble()
        t_asm = time.perf_counter() - t0
        us = _time_apply(op, nrhs, steps)
        row = {"leaf_level": leaf, "chunk_cols": 128, "apply_us": us, "assembly_s": t_asm,
               "op_bytes": op.info.op_bytes}
        table.append(row)
        if best is None or us < best["apply_us"]:
            best = dict(row)
        del op
    if best is not None and nrhs == 1:
        for ch in chunks:
            if ch == 128:
                continue
            op = Operator(space, q=q, eta=eta, leaf_level=best["leaf_level"], chunk_cols=ch)
            us = _time_apply(op, nrhs, steps)
            table.append({"leaf_level": best["leaf_level"], "chunk_cols": ch, "apply_us": us})
            if us < best["apply_us"]:
                best.update({"chunk_cols": ch, "apply_us": us})
            del op
    out = {"leaf_level": best["leaf_level"] if best else None, "chunk_cols": best["chunk_cols"] if best else None,
           "apply_us": best["apply_us"] if best else None, "table": table}
    if cache:
        data = {}
        if os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
        data[key] = out
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return out
