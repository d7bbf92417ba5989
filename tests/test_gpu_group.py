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
