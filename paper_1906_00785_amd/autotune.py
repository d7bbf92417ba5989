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


def cache_key(space, q: int, eta: float, nrhs: int, far_eval: bool, kappa_adm: float) -> str:
    """Everything that changes the partition or the kernels' work: the geometry and its
    parameters, level, degree, knot repetition, kernel and wavenumber (with its
    admissibility bound), q, eta, the number of right-hand sides and the far-field mode."""
    gp = ",".join(f"{v:.12g}" for v in space.geom.params)
    kap = complex(space.kappa) if space.kernel else 0j
    return (f"g{space.geom.kind}[{gp}]_L{space.level}_d{space.degree}_m{space.knot_repetition}_k{space.kernel}"
            f"[{kap.real:.12g},{kap.imag:.12g}]_q{q}_eta{eta}_r{nrhs}_fe{int(bool(far_eval))}_ka{kappa_adm:.12g}")


def tune(space, q: int = 5, eta: float = 1.6, nrhs: int = 1, leaf_levels=None, chunks=(128, 256, 512),
         steps: int = 20, budget_bytes: float = 16e9, cache: str | None = None, far_eval: bool = False,
         kappa_adm: float = 0.0) -> dict:
    """Returns {"leaf_level", "chunk_cols", "apply_us", "table": [...]} for the space."""
    L = space.level
    key = cache_key(space, q, eta, nrhs, far_eval, kappa_adm)
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
        op = Operator(space, q=q, eta=eta, leaf_level=leaf, assemble=False, batch_rhs=batch, far_eval=far_eval,
                      kappa_adm=kappa_adm)
        if op.info.op_bytes > budget_bytes:
            table.append({"leaf_level": leaf, "chunk_cols": 0, "skipped": f"{op.info.op_bytes/1e9:.1f} GB"})
            continue
        t0 = time.perf_counter()
        op.assemble()
        t_asm = time.perf_counter() - t0
        us = _time_apply(op, nrhs, steps)
        row = {"leaf_level": leaf, "chunk_cols": 256 if far_eval else 128, "apply_us": us, "assembly_s": t_asm,
               "op_bytes": op.info.op_bytes}
        table.append(row)
        if best is None or us < best["apply_us"]:
            best = dict(row)
        del op
    if best is not None and nrhs == 1:
        for ch in chunks:
            if ch == (256 if far_eval else 128):  # measured above
                continue
            op = Operator(space, q=q, eta=eta, leaf_level=best["leaf_level"], chunk_cols=ch, far_eval=far_eval,
                          kappa_adm=kappa_adm)
            us = _time_apply(op, nrhs, steps)
            table.append({"leaf_level": best["leaf_level"], "chunk_cols": ch, "apply_us": us})
            if us < best["apply_us"]:
                best.update({"chunk_cols": ch, "apply_us": us})
            del op
    out = {"key": key, "leaf_level": best["leaf_level"] if best else None, "chunk_cols": best["chunk_cols"] if best else None,
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
