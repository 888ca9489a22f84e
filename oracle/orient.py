"""Oracle of PC steps 2 and 3: orientation of a learned skeleton into a CPDAG.

TEST INFRASTRUCTURE ONLY: a plain, slow Python reference (numpy boolean vectors
for the premises over a third node).  Only the test
suite may use it; the product library never does, and it shares no code with
the library's orientation.

Section III-C of the paper names the three steps of PC: the skeleton (step 1,
what the rest of this oracle computes), then the v-structures found from the
separating sets (step 2), then the propagation of orientations (step 3, the
rules of Meek).  The paper gives no further detail; the readings used:

- Step 2: for every unshielded triple x - z - y (x and y not adjacent, both
  adjacent to z), if z is not in SepSet(x, y), then x -> z <- y.  All triples
  are judged on the skeleton alone, so the result does not depend on their
  order; an edge that two triples orient in opposite directions is marked
  with arrowheads at both ends (a conflict).
- Step 3: Meek's rules R1-R3 on the edges that are still undirected, with
  only directed edges (one arrowhead) as premises:
    R1  a -> b - c, a and c not adjacent               =>  b -> c
    R2  a -> c -> b and a - b                          =>  a -> b
    R3  a - b, a - c, a - d, c -> b, d -> b, c and d not adjacent  =>  a -> b
  applied in rounds: every orientation the current graph implies is found
  first, then all are applied together; an undirected edge that one round
  orients both ways gets arrowheads at both ends.  Rounds repeat until none
  orients anything.  (R4 is only needed with background knowledge.)

Output: an int8 matrix G with G[i][j] = 0 when i and j are not adjacent, 1
when they are and the edge has no arrowhead at j, 2 when it has one at j; so
i -> j is G[i][j] = 2, G[j][i] = 1, an undirected edge 1/1, a conflict 2/2.
"""

from __future__ import annotations

import numpy as np


def v_structures(adj, sepsets):
    """Step 2 on a skeleton (adj: symmetric 0/1) with sepsets {(i, j): S}
    for i < j of every non-adjacent pair.  Returns the mark matrix."""
    n = adj.shape[0]
    G = np.zeros((n, n), dtype=np.int8)
    G[adj.astype(bool)] = 1
    heads = set()  # (tail, head) orientations implied by the triples
    for z in range(n):
        nb = [u for u in range(n) if adj[z, u]]
        for ai in range(len(nb)):
            for bi in range(ai + 1, len(nb)):
                x, y = nb[ai], nb[bi]
                if adj[x, y]:
                    continue
                if z not in sepsets[(min(x, y), max(x, y))]:
                    heads.add((x, z))
                    heads.add((y, z))
    for (t, h) in heads:
        G[t, h] = 2
    return G


def meek_round(G):
    """Orientations (a, b) meaning a -> b implied by R1-R3 on G.  The
    premises over the third node c are boolean vectors over all nodes:
    D[c, a] is "c -> a", U[a, c] is "a - c"."""
    n = G.shape[0]
    adj = G > 0
    D = (G == 2) & (G.T == 1)
    U = (G == 1) & (G.T == 1)
    found = set()
    for a in range(n):
        for b in range(n):
            if a == b or not U[a, b]:
                continue
            # R1: some c -> a with c, b not adjacent orients a -> b
            r1 = D[:, a] & ~adj[:, b]
            r1[b] = False
            if r1.any():
                found.add((a, b))
                continue
            # R2: a -> c -> b orients a -> b
            if (D[a, :] & D[:, b]).any():
                found.add((a, b))
                continue
            # R3: a - c -> b and a - d -> b with c, d not adjacent orients a -> b
            cs = np.flatnonzero(U[a, :] & D[:, b])
            if any(not adj[c, d] for i, c in enumerate(cs) for d in cs[i + 1:]):
                found.add((a, b))
    return found


def orient(adj, sepsets):
    """Steps 2 and 3: the CPDAG mark matrix of a skeleton and its sepsets."""
    G = v_structures(adj, sepsets)
    while True:
        found = meek_round(G)
        if not found:
            return G
        for (a, b) in found:
            G[a, b] = 2
            if (b, a) not in found:
                G[b, a] = 1
