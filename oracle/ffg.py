"""Oracle for the search-difficulty analysis of section V.B (test
infrastructure only): fitness flow graph over a measured tune space and the
proportion of PageRank centrality.

Neighbours: configurations that differ in exactly one tunable (brute force
over all pairs).  Edges point to strictly better neighbours.  PageRank with
damping d and uniform teleportation, the rank of nodes without out-edges
spread uniformly, obtained here by a direct dense linear solve of
(I - d M) x = (1 - d)/N 1 with the column-stochastic transition matrix M --
a different method from the library's power iteration.
"""
import numpy as np


def neighbours(configs):
    c = np.asarray(configs)
    diff = (c[:, None, :] != c[None, :, :]).sum(axis=2)
    return diff == 1


def ffg_pagerank(configs, fitness, damping=0.85):
    f = np.asarray(fitness, dtype=np.float64)
    n = f.size
    nb = neighbours(configs)
    edge = nb & (f[None, :] < f[:, None])          # edge[u, v]: u -> v, v better
    outdeg = edge.sum(axis=1)
    m = np.zeros((n, n))
    for u in range(n):
        if outdeg[u]:
            m[edge[u], u] = 1.0 / outdeg[u]
        else:
            m[:, u] = 1.0 / n
    x = np.linalg.solve(np.eye(n) - damping * m, np.full(n, (1.0 - damping) / n))
    return x, outdeg == 0


def proportion_of_centrality(configs, fitness, p_values, damping=0.85):
    f = np.asarray(fitness, dtype=np.float64)
    pr, is_min = ffg_pagerank(configs, f, damping)
    f_opt = f.min()
    tot = pr[is_min].sum()
    return [float(pr[is_min & (f <= p * f_opt)].sum() / tot) for p in p_values]
