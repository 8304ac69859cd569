"""Logical race freedom of the pipelined persistent solve, checked on the CPU.

The persistent kernel runs the job list of the host scheduler: every job
waits on the counters of the jobs whose results it reads, then publishes its
own counter.  This test rebuilds, from the real job list, the happens-before
graph that those waits create and the states each job reads and writes (as
the device code of the pipeline does them), and checks that every pair of
conflicting accesses (two writes, or a write and a read, of one state by two
different jobs) is ordered by the graph: then no timing of the jobs on the
device can make a read see a state from before its producer's write, or make
a write clobber a state that a job still reads.  The ordering of the memory
operations themselves (release / acquire sequences) is checked separately in
test_release_sequence.py.

Modelled per job (type, k, n, g) of one problem (Ns slices, K iterations):
  whole coarse C(k,n): waits C(k,n-1), F(k-1,n), C(k-1,n); reads U(k,n-1),
      G(k-1,n), F(k-1,n), U(k-1,n); writes U(k,n), G(k,n), part(k-1,n)
  stage 1 of C(k,n), group g: waits C(k,n-1); reads U(k,n-1); writes P1(k,g),
      then counts in
  midpoint of a split C(k,n) (the last stage-1 job to count in): after every
      stage-1 job, reads every P1(k,.); writes Y(k)
  stage 2 of C(k,n), group g: waits C(k,n-1); reads U(k,n-1); then waits the
      midpoint and reads Y(k); writes P2(k,g), then counts in
  finish of a split C(k,n) (the last stage-2 job to count in): after every
      stage-2 job, waits F(k-1,n), C(k-1,n); reads every P2(k,.), G(k-1,n),
      F(k-1,n), U(k-1,n); writes U(k,n), G(k,n), part(k-1,n)
  fine slices n..n+g-1 of level k: waits C(k, n+g-2); reads U(k, n-1..n+g-2);
      writes F(k, n..n+g-1)
  copy (exact slice n <= k): waits C(k-1,n) and (n = k) F(k-1,k); reads
      U(k-1,n) or F(k-1,k), G(k-1,n), U(k-1,n); writes U(k,n), G(k,n),
      part(k-1,n)
  with a tolerance, the job completing C(k,Ns) also reads every part(k-1,.)
      and waits for the copy jobs of level k.
U(k,0) is u0 = U(0,0), written by the host before the launch.
"""
import pytest

from paper_1303_6615_amd import binding
from paper_1303_6615_amd.build import LIB_PATH

COARSE, FINE, STAGE1, STAGE2, COPY = 0, 1, 2, 3, 4


class Graph:
    def __init__(self):
        self.preds = []
        self.acc = {}          # location -> [(node, owner, is_write)]

    def node(self):
        self.preds.append([])
        return len(self.preds) - 1

    def edge(self, a, b):
        self.preds[b].append(a)

    def access(self, node, owner, loc, write):
        self.acc.setdefault(loc, []).append((node, owner, write))

    def races(self, limit=5):
        """Conflicting access pairs not ordered by the graph."""
        n = len(self.preds)
        indeg = [len(p) for p in self.preds]
        succ = [[] for _ in range(n)]
        for b, ps in enumerate(self.preds):
            for a in ps:
                succ[a].append(b)
        order = [v for v in range(n) if indeg[v] == 0]
        for v in order:
            for w in succ[v]:
                indeg[w] -= 1
                if indeg[w] == 0:
                    order.append(w)
        assert len(order) == n, "the wait graph has a cycle"
        anc = [0] * n
        for v in order:
            a = 0
            for p in self.preds[v]:
                a |= anc[p] | (1 << p)
            anc[v] = a

        def before(a, b):
            return a == b or (anc[b] >> a) & 1

        out = []
        for loc, lst in self.acc.items():
            for i, (na, oa, wa) in enumerate(lst):
                for nb, ob, wb in lst[i + 1:]:
                    if oa == ob or not (wa or wb):
                        continue
                    if not (before(na, nb) or before(nb, na)):
                        out.append((loc, oa, ob))
                        if len(out) >= limit:
                            return out
        return out


def build_graph(jobs, Ns, K, tol, plant_missing_copy_wait=False):
    """Happens-before graph and accesses of one problem's job list."""
    g = Graph()
    host_in, host_out = g.node(), g.node()
    g.access(host_in, "host", ("U", 0, 0), True)
    split = any(j[0] == STAGE1 for j in jobs)
    groups = max([j[3] for j in jobs if j[0] == STAGE1], default=-1) + 1
    start, end = {}, {}
    for j in jobs:
        start[j], end[j] = g.node(), g.node()
        g.edge(host_in, start[j])
        g.edge(start[j], end[j])
        g.edge(end[j], host_out)
    fin, mid = {}, {}
    if split:
        for j in jobs:
            if j[0] == STAGE1 and (j[1], j[2]) not in fin:
                fin[(j[1], j[2])] = g.node()
                mid[(j[1], j[2])] = g.node()
                g.edge(fin[(j[1], j[2])], host_out)
                g.edge(mid[(j[1], j[2])], host_out)
    comp, fine_comp = {}, {}
    for j in jobs:
        t, k, n, gg = j
        if t in (COARSE, COPY):
            comp[(k, n)] = end[j]
        elif t == FINE:
            for s in range(gg):
                fine_comp[(k, n + s)] = end[j]
    comp.update(fin)

    def U(k, n):
        return ("U", 0, 0) if n == 0 else ("U", k, n)

    def wait_copies(k, n, node):
        if tol > 0 and k >= 1 and n == Ns and not plant_missing_copy_wait:
            for m in range(1, min(k, Ns - 1) + 1):
                g.edge(comp[(k, m)], node)

    def read_parts(k, n, node, owner):
        if tol > 0 and k >= 1 and n == Ns:
            for m in range(1, Ns + 1):
                g.access(node, owner, ("part", k - 1, m), False)

    def finish(k, n, node, owner):
        # reads of the correction and the residual, writes of the step's results
        if k >= 1:
            for loc in (("G", k - 1, n), ("F", k - 1, n), U(k - 1, n)):
                g.access(node, owner, loc, False)
            g.access(node, owner, ("part", k - 1, n), True)
        g.access(node, owner, U(k, n), True)
        g.access(node, owner, ("G", k, n), True)
        read_parts(k, n, node, owner)

    for j in jobs:
        t, k, n, gg = j
        s, e = start[j], end[j]
        if t == COARSE:
            if n > 1:
                g.edge(comp[(k, n - 1)], s)
            if k >= 1:
                g.edge(fine_comp[(k - 1, n)], s)
                g.edge(comp[(k - 1, n)], s)
            wait_copies(k, n, s)
            g.access(s, j, U(k, n - 1), False)
            finish(k, n, e, j)
        elif t == STAGE1:
            if n > 1:
                g.edge(comp[(k, n - 1)], s)
            g.access(s, j, U(k, n - 1), False)
            g.access(e, j, ("P1", k, gg), True)
            g.edge(e, mid[(k, n)])
        elif t == STAGE2:
            if n > 1:
                g.edge(comp[(k, n - 1)], s)
            g.access(s, j, U(k, n - 1), False)
            after_mid = g.node()
            g.edge(s, after_mid)
            g.edge(mid[(k, n)], after_mid)
            g.edge(after_mid, e)
            g.access(after_mid, j, ("Y", k), False)
            g.access(e, j, ("P2", k, gg), True)
            g.edge(e, fin[(k, n)])
        elif t == FINE:
            last = n + gg - 2 if gg > 1 else n - 1
            if last >= 1:
                g.edge(comp[(k, last)], s)
            for x in range(gg):
                g.access(s, j, U(k, n - 1 + x), False)
                g.access(e, j, ("F", k, n + x), True)
        elif t == COPY:
            if n == k:
                g.edge(fine_comp[(k - 1, n)], s)
            g.edge(comp[(k - 1, n)], s)
            wait_copies(k, n, s)
            g.access(s, j, U(k - 1, n) if n < k else ("F", k - 1, k), False)
            g.access(s, j, ("G", k - 1, n), False)
            g.access(s, j, U(k - 1, n), False)
            g.access(e, j, U(k, n), True)
            g.access(e, j, ("G", k, n), True)
            g.access(e, j, ("part", k - 1, n), True)
            read_parts(k, n, e, j)
    for (k, n), m in mid.items():
        for x in range(groups):
            g.access(m, ("mid", k, n), ("P1", k, x), False)
        g.access(m, ("mid", k, n), ("Y", k), True)
    for (k, n), f in fin.items():
        owner = ("finish", k, n)
        if k >= 1:
            g.edge(fine_comp[(k - 1, n)], f)
            g.edge(comp[(k - 1, n)], f)
        wait_copies(k, n, f)
        for x in range(groups):
            g.access(f, owner, ("P2", k, x), False)
        finish(k, n, f, owner)
    for n in range(1, Ns + 1):
        g.access(host_out, "host", U(K, n), False)
    for k in range(K):
        for n in range(1, Ns + 1):
            g.access(host_out, "host", ("part", k, n), False)
    return g


@pytest.fixture(scope="module")
def L():
    import os
    if not os.path.exists(LIB_PATH):
        pytest.fail("libaparareal.so not built (run python -m paper_1303_6615_amd.build)")
    return binding.lib()


CASES = [  # N, T, Ns, K, dt, M, split, group, fine group, tol
    (64, 1.0, 16, 5, 0.0005, 16, -1, 0, 1, 0.0), (256, 2.0, 64, 8, 0.0005, 32, -1, 0, 1, 0.0),
    (512, 0.1, 16, 8, 0.005, 32, 1, 0, 1, 0.0), (512, 0.1, 16, 8, 0.005, 32, 1, 0, 2, 0.0),
    (256, 2.0, 64, 8, 0.0005, 32, 0, 0, 5, 0.0), (128, 0.7, 7, 3, 0.1, 2, 1, 0, 4, 0.0),
    (64, 1.0, 4, 6, 0.05, 9, 1, 1, 3, 0.0), (1024, 1.0, 40, 10, 0.0001, 64, -1, 0, 1, 0.0),
    (512, 0.1, 16, 8, 0.005, 32, 1, 0, 1, 1e-6), (256, 1.0, 12, 8, 0.001, 32, 0, 0, 5, 1e-6),
    (64, 1.0, 5, 7, 0.05, 9, 1, 2, 4, 1e-3), (128, 1.0, 3, 6, 0.05, 9, 0, 0, 2, 1e-3),
]


@pytest.mark.parametrize("N,T,Ns,K,dt,M,split,group,fg,tol", CASES)
def test_every_conflicting_access_is_ordered(L, N, T, Ns, K, dt, M, split, group, fg, tol):
    jobs = binding.pipeline_schedule(N, T, Ns, K, dt, M, split=split, group=group, fine_group=fg, tol=tol)
    g = build_graph(jobs, Ns, K, tol)
    assert g.races() == []


def test_checker_finds_the_unordered_residual_read(L):
    # without the waits on the copy jobs, the tolerance check of C(k, Ns)
    # reads residual parts that copy jobs of level k may not have written yet
    N, T, Ns, K, dt, M, tol = 512, 0.1, 16, 8, 0.005, 32, 1e-6
    jobs = binding.pipeline_schedule(N, T, Ns, K, dt, M, split=1, fine_group=1, tol=tol)
    bad = build_graph(jobs, Ns, K, tol, plant_missing_copy_wait=True).races()
    assert bad and all(r[0][0] == "part" for r in bad)


def test_checker_finds_a_dropped_wait():
    # a write and a read of one state by two jobs: unordered until an edge
    # (a wait) orders them
    g2 = Graph()
    a, b = g2.node(), g2.node()
    g2.access(a, "x", ("U", 0, 1), True)
    g2.access(b, "y", ("U", 0, 1), False)
    assert g2.races() == [(("U", 0, 1), "x", "y")]
    g2.edge(a, b)
    assert g2.races() == []


def test_batched_schedules_with_tolerances_are_race_free(L):
    probs = [(512, 0.1, 16, 8, 0.005, 32, 1e-6), (256, 1.0, 9, 8, 0.001, 16, 0.0),
             (128, 0.5, 5, 6, 0.01, 9, 1e-3)]
    jobs = binding.pipeline_schedule_batch(probs, split=1, fine_group=2)
    for i, (N, T, Ns, K, dt, M, tol) in enumerate(probs):
        mine = [j[1:] for j in jobs if j[0] == i]
        assert build_graph(mine, Ns, K, tol).races() == []
