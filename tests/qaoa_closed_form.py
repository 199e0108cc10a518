"""Closed form of one QAOA layer for MaxCut on unweighted graphs (test
infrastructure: an independent pin for the oracle and, at sizes the oracle
cannot hold, for the device path)."""
import math


def qaoa1_zz_closed_form(edges, n, u, v, theta_cost, theta_mix):
    """<Z_u Z_v> after one QAOA layer on |+>^n for an unweighted graph, from
    the closed form of Wang, Hadfield, Jiang and Rieffel (Phys. Rev. A 97,
    022304, 2018, Theorem 1) for C_uv = (1 - Z_u Z_v) / 2 with
    |psi> = exp(-i beta B) exp(-i gamma C) |+>^n, B = sum_j X_j:
      <C_uv> = 1/2 + sin(4 beta) sin(gamma) (cos^du(gamma) + cos^dv(gamma)) / 4
               - sin^2(2 beta) cos^(du + dv - 2 f)(gamma) (1 - cos^f(2 gamma)) / 4,
    du = deg(u) - 1, dv = deg(v) - 1, f = triangles through (u, v).  The
    circuit's cost layer exp(-i t Z_u Z_v / 2) per edge is exp(-i gamma C) up
    to a phase with gamma = -t, and RX(t) = exp(-i t X / 2) gives beta = t / 2."""
    adj = {q: set() for q in range(n)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    du, dv = len(adj[u]) - 1, len(adj[v]) - 1
    f = len(adj[u] & adj[v])
    g, bt = -theta_cost, theta_mix / 2
    c = (0.5 + 0.25 * math.sin(4 * bt) * math.sin(g) * (math.cos(g) ** du + math.cos(g) ** dv)
         - 0.25 * math.sin(2 * bt) ** 2 * math.cos(g) ** (du + dv - 2 * f) * (1 - math.cos(2 * g) ** f))
    return 1.0 - 2.0 * c
