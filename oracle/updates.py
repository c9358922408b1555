"""Index updates of the RoarGraph oracle (TEST INFRASTRUCTURE ONLY): insertion
through the saved bipartite graph and deletion by tombstones (Sec. 6,
"Update in RoarGraph").  Plain Python over the oracle's C primitives
(canonical FP64 distance, beam search, AcquireNeighbors); nothing here is
fast and nothing is shared with the library.

Readings of the passage (the paper gives it in prose only):

* A batch of insertions first searches every new vector v on the index as
  it stood when the batch began (queue length L, the build's L by default;
  the final queue in (delta, id) order).  The graph updates then run for
  the vectors in input order; v gets id n, n+1, ... in that order.
* "Connected to a query node": b is the pivot of some training query t
  (edge b -> t) or b is in N_out(t) for some t.  b is the first node of v's
  queue that is connected; among the query nodes connected to b, q is the
  one nearest to v by (delta(v, t), t).
* The sub-bipartite graph N_out(q) u {q, v} is projected with v as pivot,
  exactly as Algorithm 2 treats a pivot: the candidates N_out(q) ranked by
  (delta(v, c), c) and cut to L, then AcquireNeighbors with fill to m_pj.
  In that small projected graph every selected p gains the edge p -> v.
* Merging into the index: v's row is its selection; each selected p, in
  selection order, reconsiders its row as Algorithm 2's reverse step does:
  row(p) <- AcquireNeighbors(p, row(p) u {v}, M) with fill (a row with room
  simply gains v; a full row keeps the M best by the selection rule, which
  may drop v or an old neighbour).  If no p kept v, v gets one in-edge by
  the build's repair rule: from the first node of its queue with a free
  slot, else the first node in BFS order from the entry (neighbours in
  ascending id) with a free slot.
* At the end of the call, every node the entry no longer reaches (an old
  neighbour dropped above can lose its last in-edge) gets one in-edge, in
  ascending id, from the first node in BFS order with a free slot, and the
  BFS continues from it.
* Finally v is appended to N_out(q).  If no node of the queue is connected,
  v's candidates are its queue itself and N_out is not changed.
* Tombstones: a deleted node stays in the graph and in every queue (it
  routes) but is skipped when the k results are taken from the final queue.
"""
from __future__ import annotations

import numpy as np

from . import NONE, acquire, dist, search as _search


class Updatable:
    """Graph, bipartite graph and vectors that the update procedures change."""

    def __init__(self, rows, entry, M, L, X, T, pivot, nout, m_pj=None):
        self.X = np.ascontiguousarray(X, dtype=np.float32)
        self.T = np.ascontiguousarray(T, dtype=np.float32)
        self.rows = [sorted(map(int, r)) for r in rows]
        self.entry = int(entry)
        self.M, self.L = int(M), int(L)
        self.m_pj = int(m_pj) if m_pj else self.M // 2   # ceil((M-1)/2), the build's default
        self.pivot = [int(p) for p in pivot]
        self.nout = [list(map(int, r)) for r in nout]
        self.deleted = set()

    @classmethod
    def from_graph(cls, G, X, T):
        """State of a finished oracle build (Graph) over base X and training T."""
        return cls(G.rows("final"), G.entry, G.M, G.L, X, T, G.pivot, G.nout)

    @property
    def n(self):
        return len(self.rows)

    def csr(self):
        off = np.zeros(self.n + 1, np.int64)
        off[1:] = np.cumsum([len(r) for r in self.rows])
        idx = np.array([u for r in self.rows for u in r], np.uint32)
        return off, idx

    def connected(self, b):
        """Query nodes joined to base node b in the bipartite graph, either way."""
        return [t for t in range(len(self.pivot)) if self.pivot[t] == b or b in self.nout[t]]

    def bfs_order(self):
        seen = np.zeros(self.n, bool)
        seen[self.entry] = True
        order = [self.entry]
        h = 0
        while h < len(order):
            for w in self.rows[order[h]]:
                if not seen[w]:
                    seen[w] = True
                    order.append(w)
            h += 1
        return order

    def insert(self, V, L=None):
        V = np.ascontiguousarray(V, dtype=np.float32).reshape(-1, self.X.shape[1])
        L = int(L or self.L)
        off, idx = self.csr()
        queues, _, _, _, _ = _search(self.X, off, idx, self.entry, V, L, L)
        first = self.n
        self.X = np.concatenate([self.X, V])
        for i in range(len(V)):
            v = first + i
            queue = [int(u) for u in queues[i] if u != NONE]
            b = next((u for u in queue if self.connected(u)), None)
            if b is None:
                q, cand = None, queue
            else:
                q = min(self.connected(b), key=lambda t: (dist(V[i], self.T[t]), t))
                cand = list(self.nout[q])
            ranked = sorted(set(cand) - {v}, key=lambda c: (dist(V[i], self.X[c]), c))[:L]
            sel = [int(p) for p in acquire(self.X, v, np.array(ranked, np.uint32), self.m_pj, True)]
            self.rows.append(sorted(sel))
            took = False
            for p in sel:
                kept = acquire(self.X, p, np.array(self.rows[p] + [v], np.uint32), self.M, True)
                self.rows[p] = sorted(int(u) for u in kept)
                took = took or v in self.rows[p]
            if not took:
                r = next((u for u in queue if len(self.rows[u]) < self.M), None)
                if r is None:
                    r = next((u for u in self.bfs_order() if len(self.rows[u]) < self.M), None)
                if r is None:
                    raise RuntimeError("insert: no node with a free slot")
                self.rows[r].append(v)
            if q is not None:
                self.nout[q].append(v)
        self.repair()
        return np.arange(first, first + len(V), dtype=np.uint32)

    def repair(self):
        """Reconnect every node the entry does not reach (see the module text)."""
        seen = np.zeros(self.n, bool)
        seen[self.entry] = True
        order = [self.entry]
        h = 0

        def bfs(h):
            while h < len(order):
                for w in self.rows[order[h]]:
                    if not seen[w]:
                        seen[w] = True
                        order.append(w)
                h += 1
            return h

        h = bfs(h)
        for u in range(self.n):
            if seen[u]:
                continue
            r = next((x for x in order if len(self.rows[x]) < self.M), None)
            if r is None:
                raise RuntimeError("insert: no node with a free slot")
            self.rows[r] = sorted(self.rows[r] + [u])
            seen[u] = True
            order.append(u)
            h = bfs(h)

    def delete(self, ids):
        for u in ids:
            self.deleted.add(int(u))

    def search(self, Q, k, L):
        """Beam search; the k results skip deleted nodes of the final queue."""
        off, idx = self.csr()
        Leff = max(k, L)
        ids, ds, _, _, _ = _search(self.X, off, idx, self.entry, Q, Leff, L)
        out_i = np.full((len(Q), k), NONE, np.uint32)
        out_d = np.full((len(Q), k), np.inf)
        for r in range(len(Q)):
            keep = [(u, x) for u, x in zip(ids[r], ds[r]) if u != NONE and int(u) not in self.deleted][:k]
            for j, (u, x) in enumerate(keep):
                out_i[r, j], out_d[r, j] = u, x
        return out_i, out_d
