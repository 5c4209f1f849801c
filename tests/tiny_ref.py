"""Brute-force label propagation on tiny dense graphs (test helper, n <= 12).

An independent, deliberately naive restatement of the sequential method of
Algorithm 1 (Section 4.2): the graph is a dense weight matrix plus a dense
adjacency matrix, the active set is a Python set, per-label weights are
collected in a dict and the winner is taken with max() over (weight, -label).
It shares nothing with the C oracle and exists only to cross-check it
exhaustively on small inputs.
"""


def dense(n, offsets, indices, weights=None):
    W = [[0] * n for _ in range(n)]
    adj = [[False] * n for _ in range(n)]
    for i in range(n):
        for k in range(int(offsets[i]), int(offsets[i + 1])):
            j = int(indices[k])
            W[i][j] += 1 if weights is None else int(weights[k])
            adj[i][j] = True
    return W, adj


def lpa_dense(W, adj, order=None, tau=0.05, max_iters=20, prune=True, tie=None):
    """tie(c, v): key of label c among equally heavy labels at vertex v (the
    smallest key wins); None = the label id itself (strict LPA)."""
    n = len(W)
    order = list(range(n)) if order is None else [int(v) for v in order]
    label = list(range(n))
    active = set(range(n))
    history = []
    converged = False
    for _ in range(max_iters):
        moved = 0
        for v in order:
            if prune and v not in active:
                continue
            active.discard(v)
            nbrs = [j for j in range(n) if j != v and adj[v][j]]
            if not nbrs:
                continue
            tally = {}
            for j in nbrs:
                tally[label[j]] = tally.get(label[j], 0) + W[v][j]
            top = max(tally.values())
            best = min((c for c, x in tally.items() if x == top), key=lambda c: c if tie is None else tie(c, v))
            if best != label[v]:
                label[v] = best
                moved += 1
                active.update(nbrs)
        history.append(moved)
        if moved / n <= tau:
            converged = True
            break
    return label, history, converged
