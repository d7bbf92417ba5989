"""GPU: grouped launches over many uneven operators and captured launch sequences, against
the oracle at the batched workload's own levels.

Instances: one of the batched uneven workload's seeded draws for every combination of
geometry (ellipsoid, torus), PDE (Laplace with the coupling evaluated on the fly, Helmholtz
with stored blocks) and level 2..5, each with its own degree, wavenumber and 1..16 columns.

Bar: every grouped output column and every graph replay within 1e-11 (max-norm, relative
to the largest oracle entry) of the oracle's H^2 product with the same q, eta and leaf
level.  Level 2: the oracle's full product.  Levels 3 to 5: the oracle's product on sampled
rows (near and far), plus the far field at every row (the oracle's far pipeline is cheap;
the near part of those rows comes from the exported near field, whose sampled rows the
first comparison pins; the oracle's full near field at level 3 takes minutes of serial
host time).  Replays run with eager work between them that changes the
inputs in place, and each replay is compared with the oracle on the inputs of that moment.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11
Q, ETA = W.CONFIGS[3]["q"], W.CONFIGS[3]["eta"]


@pytest.fixture(scope="module")
def B():
    import paper_1906_00785_amd as B

    return B


def subset():
    """Indices into the 512 seeded instances: the first of each (geometry, PDE, level)."""
    insts = W.c3_instances(512)
    sel = {}
    for k, it in enumerate(insts):
        sel.setdefault((it["geom"], it["pde"], it["level"]), k)
    assert len(sel) == 16
    return [(k, insts[k]) for _, k in sorted(sel.items())]


class Member:
    """One instance: the GPU operator, its seeded input columns and the oracle operator."""

    def __init__(self, B, orc, k, it):
        L = it["level"]
        self.k, self.it, self.L, self.leaf = k, it, L, max(L - 2, 0)
        self.cplx = bool(it["pde"])
        print(f"[group] instance {k}: geom {it['geom']} {tuple(round(v, 3) for v in it['params'])} L={L} "
              f"d={it['degree']} pde={it['pde']} kappa={it['kappa']:.3f} ncols={len(it['sources'])}", flush=True)
        g = B.Geometry(it["geom"], it["params"])
        self.s = B.Space(g, it["pde"], it["kappa"], degree=it["degree"], level=L)
        self.A = B.Operator(self.s, q=Q, eta=ETA, leaf_level=self.leaf, far_eval=it["pde"] == 0)
        self.N = self.s.ndof
        xh = W.random_vector(W.rng(3, 200 + k), self.N, is_complex=self.cplx, ncols=len(it["sources"]))
        self.x = torch.from_numpy(np.ascontiguousarray(xh.T).reshape(len(it["sources"]), self.N)).cuda()
        So = orc.Space(it["geom"], list(it["params"]), it["pde"], it["kappa"], degree=it["degree"], level=L)
        self.full = L <= 2
        self.Ho = orc.H2(So, q=Q, eta=ETA, leaf=self.leaf, assemble_near=self.full)
        if not self.full:
            self.rows = W.sample_rows(3, self.N, 6)
            self.Ho.assemble_near_rows(self.rows)
            self.near = self.A.export_near()

    def check(self, x, y, what):
        """Columns of y (ncols, N) against the oracle's product of the columns of x."""
        xs, ys = x.cpu().numpy(), y.cpu().numpy()
        for c in range(xs.shape[0]):
            if self.full:
                yo = self.Ho.apply(xs[c])
                err = np.max(np.abs(ys[c] - yo)) / np.max(np.abs(yo))
            else:
                yo = self.Ho.apply_rows(xs[c], self.rows)
                err = np.max(np.abs(ys[c][self.rows] - yo)) / np.max(np.abs(yo))
                rowptr, col, val = self.near
                yn = np.add.reduceat(val * xs[c][col], rowptr[:-1])
                yf = self.Ho.apply_rows(xs[c], np.arange(self.N, dtype=np.int64), far=True, near=False)
                err = max(err, np.max(np.abs(ys[c] - yn - yf)) / np.max(np.abs(ys[c])))
            assert err <= TOL, (what, self.k, c, err)


@pytest.fixture(scope="module")
def members(B, orc):
    return [Member(B, orc, k, it) for k, it in subset()]


def test_subset_covers_the_workload(members):
    got = {(m.it["geom"], m.it["pde"], m.L) for m in members}
    assert got == {(g, p, L) for g in (1, 2) for p in (0, 1) for L in (2, 3, 4, 5)}
    assert {m.it["degree"] for m in members} == {1, 2}


def test_group_matches_oracle(B, members):
    for pde in (0, 1):
        grp = [m for m in members if m.it["pde"] == pde]
        ys = [torch.empty_like(m.x) for m in grp]
        G = B.Group([m.A for m in grp], [m.x for m in grp], ys)
        G.apply()
        for m, y in zip(grp, ys):
            m.check(m.x, y, f"grouped pde={pde}")
            # the operator's own apply computes the same columns (same per-column kernels)
            assert torch.equal(y, m.A.apply(m.x))


def test_graph_replays_match_oracle(B, members):
    xs = [m.x.clone() for m in members]
    ys = [torch.empty_like(x) for x in xs]
    groups = [B.Group([members[i].A for i in sel], [xs[i] for i in sel], [ys[i] for i in sel])
              for sel in ([i for i, m in enumerate(members) if m.it["pde"] == p] for p in (0, 1))]
    m0 = members[0]
    x1 = torch.from_numpy(W.random_vector(W.rng(3, 300), m0.N, is_complex=m0.cplx)).cuda()
    y1 = torch.empty_like(x1)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = B.Graph()
        with graph:
            for G in groups:
                G.apply()
            m0.A.apply(x1, out=y1)
        for rep in range(3):
            # eager work between replays changes the inputs in place
            for x in xs:
                x.mul_(1.0 + 0.25 * rep)
                x.add_(0.125 * (rep + 1))
            x1.add_(0.5)
            graph.launch()
            stream.synchronize()
            print(f"[group] graph replay {rep}", flush=True)
            for m, x, y in zip(members, xs, ys):
                m.check(x, y, f"replay {rep}")
            m0.check(x1.reshape(1, -1), y1.reshape(1, -1), f"replay {rep} single apply")
    stream.synchronize()


def test_instances_through_many_rhs_kernels(B, members):
    """The instances with several columns planned with batch_rhs = their column count (the
    many-RHS slab kernels, FP64), per instance and in a graph of per-instance applies with
    eager work between the replays: every column against the oracle."""
    sel = [m for m in members if m.x.shape[0] > 1 and m.it["pde"] == 1][:4] + \
          [m for m in members if m.x.shape[0] > 1 and m.it["pde"] == 0][:4]
    ops = []
    for m in sel:
        print(f"[group-batched] instance {m.k}: L={m.L} pde={m.it['pde']} ncols={m.x.shape[0]}", flush=True)
        ops.append(B.Operator(m.s, q=Q, eta=ETA, leaf_level=m.leaf, batch_rhs=m.x.shape[0]))
    for m, A in zip(sel, ops):
        m.check(m.x, A.apply(m.x), "many-RHS kernels")
    xs = [m.x.clone() for m in sel]
    ys = [torch.empty_like(x) for x in xs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = B.Graph()
        with graph:
            for A, x, y in zip(ops, xs, ys):
                A.apply(x, out=y)
        for rep in range(2):
            for x in xs:
                x.mul_(1.0 + 0.5 * rep)
            graph.launch()
            stream.synchronize()
            for m, x, y in zip(sel, xs, ys):
                m.check(x, y, f"many-RHS graph replay {rep}")
    stream.synchronize()
