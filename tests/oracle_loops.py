"""Loop-form re-evaluation of the Allegro energy for tiny inputs (test helper).

Written independently of the vectorised oracle, in the other form that the
paper's equations allow: per ordered pair, per neighbour k, per path, with the
unfused coupling tensors and the tensor product taken *inside* the neighbour
sum (the left-hand side of Eq. tp), in plain Python floats.  Agreement with the
oracle pins its indexing (strided components, segment grouping, path fusion,
factorisation of the neighbour sum, and for deeper models the parity blocks
of the strided layout and the per-irrep mixing).
"""
import math

import numpy as np

from oracle import cg
from oracle.neighbors import neighbor_list


def _silu(v):
    return [a / (1.0 + math.exp(-a)) for a in v]


def _matvec(x, W):
    W = np.asarray(W, dtype=np.float64)
    return [sum(x[k] * W[k, c] for k in range(len(x))) for c in range(W.shape[1])]


def _mlp(x, Ws):
    for k, W in enumerate(Ws):
        x = _matvec(x, W)
        if k < len(Ws) - 1:
            x = _silu(x)
    return x


def _sh(v):
    x, y, z = v
    s3, s15, s5 = math.sqrt(3), math.sqrt(15), math.sqrt(5)
    out = [1.0, s3 * y, s3 * z, s3 * x, s15 * x * y, s15 * y * z, s5 / 2 * (3 * z * z - 1),
           s15 * x * z, s15 / 2 * (x * x - y * y)]
    c70, c105, c42, c7 = math.sqrt(70) / 4, math.sqrt(105), math.sqrt(42) / 4, math.sqrt(7) / 2
    out += [c70 * y * (3 * x * x - y * y), c105 * x * y * z, c42 * y * (5 * z * z - 1),
            c7 * z * (5 * z * z - 3), c42 * x * (5 * z * z - 1), c105 / 2 * z * (x * x - y * y),
            c70 * x * (x * x - 3 * y * y)]
    return out


def energy(mc, w, sysm):
    pos, Z = np.asarray(sysm.pos), np.asarray(sysm.species)
    L = np.where(np.asarray(sysm.pbc) != 0, np.asarray(sysm.cell, dtype=float), 0.0)
    I, J, S = neighbor_list(pos, sysm.cell, sysm.pbc, mc.r_cut, n_local=sysm.n_local, species=Z,
                            pair_cutoffs=mc.pair_cutoffs)
    n, lm, nS = mc.n_tensor, mc.l_max, mc.n_species
    dim = (lm + 1) ** 2
    lof = [l for l in range(lm + 1) for _ in range(2 * l + 1)]
    paths = cg.layer_paths(lm, mc.n_layers)

    def off(l, p):   # first component of irrep (l, p): natural block, then the other parity
        return l * l + (0 if p == (-1) ** l else dim)

    def slot(c):     # mixing matrix of component c
        return lof[c] if c < dim else lm + 1 + lof[c - dim]

    def width(irreps):
        return 2 * dim if any(p != (-1) ** l for (l, p) in irreps) else dim
    edges = []
    for (i, j, s) in zip(I.tolist(), J.tolist(), S.tolist()):
        r = [(pos[j, a] - pos[i, a]) + s[a] * L[a] for a in range(3)]
        d = math.sqrt(sum(c * c for c in r))
        rc = mc.r_cut if mc.pair_cutoffs is None else mc.pair_cutoffs[Z[i]][Z[j]]
        t, p = d / rc, mc.envelope_p
        u = 1 - (p + 1) * (p + 2) / 2 * t ** p + p * (p + 2) * t ** (p + 1) - p * (p + 1) / 2 * t ** (p + 2)
        Rb = [math.sqrt(2 / rc) * math.sin(k * math.pi * d / rc) / d * u
              for k in range(1, mc.n_bessel + 1)]
        Y = _sh([c / d for c in r])[:dim]
        inp = [0.0] * (2 * nS)
        inp[Z[i]] = 1.0
        inp[nS + Z[j]] = 1.0
        x = [u * v for v in _mlp(inp + Rb, [w[f"twobody.W{k}"] for k in range(len(mc.twobody_dims))])]
        a0 = _matvec(x, w["embed0"])
        V = [[a0[lof[c] * n + q] * Y[c] for q in range(n)] for c in range(dim)]
        edges.append(dict(i=i, u=u, Y=Y, x=x, V=V))
    cn = 1.0 / math.sqrt(mc.avg_num_neighbors)
    for Lr in range(1, mc.n_layers + 1):
        final = Lr == mc.n_layers
        al = np.asarray(w[f"layer{Lr}.alpha"], dtype=np.float64)
        M = np.asarray(w[f"layer{Lr}.mix"], dtype=np.float64)
        kept = paths[Lr - 1]
        cnt = {}
        for (_, _, _, lo, po) in kept:
            cnt[(lo, po)] = cnt.get((lo, po), 0) + 1
        wk = [_matvec(e["x"], w[f"layer{Lr}.env"]) for e in edges]
        n_out = 1 if final else width([(lo, po) for (_, _, _, lo, po) in kept])
        newV = []
        for e in edges:
            T = [[0.0] * n for _ in range(n_out)]
            for (k, f) in enumerate(edges):
                if f["i"] != e["i"]:
                    continue
                for (l1, p1, l2, lo, po) in kept:
                    C = cg.coupling(l1, l2, lo)
                    raw = al[0 if p1 == (-1) ** l1 else 1, l1, l2, lo] if al.ndim == 4 else al[l1, l2, lo]
                    a = raw / math.sqrt(cnt[(lo, po)])
                    for m1 in range(2 * l1 + 1):
                        for m2 in range(2 * l2 + 1):
                            for m3 in range(2 * lo + 1):
                                cf = C[m1, m2, m3]
                                if cf == 0.0:
                                    continue
                                c1, c2, c3 = off(l1, p1) + m1, l2 * l2 + m2, off(lo, po) + m3
                                for q in range(n):
                                    T[c3][q] += a * cf * e["V"][c1][q] * cn * wk[k][l2 * n + q] * f["Y"][c2]
            if mc.channel_mix:
                Vn = [[sum(M[slot(c), v, q] * T[c][q] for q in range(n)) / math.sqrt(n) for v in range(n)]
                      for c in range(n_out)]
            else:
                Vn = T
            newV.append(Vn)
        for e, Vn in zip(edges, newV):
            h = _mlp(e["x"] + Vn[0], [w[f"layer{Lr}.mlp.W{k}"] for k in range(len(mc.latent_dims))])
            e["x"] = [(a + e["u"] * b) / math.sqrt(2) for a, b in zip(e["x"], h)]
            e["V"] = Vn
    out = []
    for e in edges:
        y = e["x"]
        for k in range(len(mc.edge_dims) + 1):
            y = _matvec(y, w[f"edge.W{k}"])
        out.append(y[0])
    return np.asarray(out)
