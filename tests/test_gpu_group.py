"""GPU: grouped launches over many uneven operators and captured launch sequences.

Bar: the grouped apply runs the same per-column computation as the one-column path, so
its output is bitwise identical to each operator's own apply (which the parity tests pin to
the oracle); every replay of a captured graph is bitwise identical to the eager result for
the inputs of that moment, with eager work between the replays.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import paper_1906_00785_amd as B

    return B


@pytest.fixture(scope="module")
def family(B):
    """24 instances of the batched uneven workload, levels capped at 3 for test time."""
    insts = W.c3_instances(24)
    ops = {0: [], 1: []}
    for k, it in enumerate(insts):
        L = min(it["level"], 3)
        print(f"[group] instance {k}: geom {it['geom']} L={L} d={it['degree']} pde={it['pde']} "
              f"nrhs={len(it['sources'])}", flush=True)
        g = B.Geometry(it["geom"], it["params"])
        s = B.Space(g, it["pde"], it["kappa"], degree=it["degree"], level=L)
        A = B.Operator(s, q=5, eta=1.6, leaf_level=max(L - 2, 0))
        x = torch.from_numpy(W.random_vector(W.rng(3, 200 + k), s.ndof, is_complex=bool(it["pde"]),
                                             ncols=len(it["sources"])).T.copy()).cuda()
        ops[it["pde"]].append((s, A, x))
    return ops


def test_group_matches_individual_applies(B, family):
    for pde, members in family.items():
        if not members:
            continue
        xs = [x for _, _, x in members]
        ys = [torch.empty_like(x) for x in xs]
        G = B.Group([A for _, A, _ in members], xs, ys)
        G.apply()
        for (s, A, x), y in zip(members, ys):
            assert torch.equal(y, A.apply(x))


def test_graph_replays_match_eager(B, family):
    members = family[1] or family[0]
    xs = [x.clone() for _, _, x in members]
    ys = [torch.empty_like(x) for x in xs]
    G = B.Group([A for _, A, _ in members], xs, ys)
    s0, A0, _ = members[0]
    x1 = torch.from_numpy(W.random_vector(W.rng(3, 300), s0.ndof, is_complex=s0.dtype == torch.complex128)).cuda()
    y1 = torch.empty_like(x1)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = B.Graph()
        with graph:
            G.apply()
            A0.apply(x1, out=y1)
        for rep in range(3):
            # eager work between replays changes the inputs in place
            for x in xs:
                x.mul_(1.0 + 0.25 * rep)
            x1.add_(0.5)
            graph.launch()
            got = [y.clone() for y in ys]
            got1 = y1.clone()
            G.apply()
            A0.apply(x1, out=y1)
            for g_, y in zip(got, ys):
                assert torch.equal(g_, y), rep
            assert torch.equal(got1, y1), rep
    stream.synchronize()


def test_instances_through_many_rhs_kernels(B):
    """Instances planned with batch_rhs = their column count: the per-instance apply (slab
    kernels) agrees with the grouped one-column launches to rounding (1e-13 relative), and
    a graph of per-instance applies replays bitwise like the eager applies, with eager work
    between the replays."""
    insts = [it for it in W.c3_instances(24) if len(it["sources"]) > 1][:6]
    ops, xs = [], []
    for k, it in enumerate(insts):
        L = min(it["level"], 3)
        print(f"[group-batched] instance {k}: geom {it['geom']} L={L} pde={it['pde']} nrhs={len(it['sources'])}",
              flush=True)
        g = B.Geometry(it["geom"], it["params"])
        s = B.Space(g, it["pde"], it["kappa"], degree=it["degree"], level=L)
        A = B.Operator(s, q=5, eta=1.6, leaf_level=max(L - 2, 0), batch_rhs=len(it["sources"]))
        ops.append(A)
        xs.append(torch.from_numpy(W.random_vector(W.rng(3, 400 + k), s.ndof, is_complex=bool(it["pde"]),
                                                   ncols=len(it["sources"])).T.copy()).cuda())
    for pde in (0, 1):
        sel = [k for k, it in enumerate(insts) if it["pde"] == pde]
        if not sel:
            continue
        ys = [torch.empty_like(xs[k]) for k in sel]
        B.Group([ops[k] for k in sel], [xs[k] for k in sel], ys).apply()
        for k, y in zip(sel, ys):
            yb = ops[k].apply(xs[k])
            assert float((yb - y).abs().max() / y.abs().max()) <= 1e-13
    ys = [torch.empty_like(x) for x in xs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = B.Graph()
        with graph:
            for A, x, y in zip(ops, xs, ys):
                A.apply(x, out=y)
        for rep in range(3):
            for x in xs:
                x.mul_(1.0 + 0.5 * rep)
            graph.launch()
            got = [y.clone() for y in ys]
            for A, x, g_ in zip(ops, xs, got):
                assert torch.equal(g_, A.apply(x)), rep
    stream.synchronize()
