"""Mesh complex K = {N, E, F, T} and integer incidence (Sec. II.C).

Orientation conventions (the paper fixes none):
  * every tet lists its vertices in ascending global id;
  * edge [a,b] with a < b is oriented a -> b; G[e, b] = +1, G[e, a] = -1;
  * face [a,b,c] with a < b < c has boundary [b,c] - [a,c] + [a,b], which gives C;
  * D[t, f] = sign(vol of the sorted tet) * (-1)^i for the face opposite local vertex i.
Edges and faces are numbered in lexicographic order of their sorted vertex tuples.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

LOCAL_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
LOCAL_FACES = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]  # face k is opposite vertex k


class Complex:
    def __init__(self, xyz: np.ndarray, tets: np.ndarray, neumann: bool = False):
        # neumann: natural boundary, every edge and node an unknown (PEC otherwise: wall edges
        # carry no E and wall nodes are grounded)
        self.neumann = neumann
        self.xyz = np.asarray(xyz, dtype=np.float64)
        T = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
        self.tets = T
        Nn, Nt = self.xyz.shape[0], T.shape[0]
        self.Nn, self.Nt = Nn, Nt

        # edges: unique sorted vertex pairs
        pairs = np.stack([T[:, [a, b]] for a, b in LOCAL_EDGES], axis=1).reshape(-1, 2)
        key = pairs[:, 0] * Nn + pairs[:, 1]
        ukey, inv = np.unique(key, return_inverse=True)
        self.edges = np.stack([ukey // Nn, ukey % Nn], axis=1)
        self.tet_edges = inv.reshape(Nt, 6)
        self.Ne = self.edges.shape[0]

        # faces: unique sorted vertex triples
        tri = np.stack([T[:, list(f)] for f in LOCAL_FACES], axis=1).reshape(-1, 3)
        fkey = (tri[:, 0] * Nn + tri[:, 1]) * Nn + tri[:, 2]
        ufkey, finv = np.unique(fkey, return_inverse=True)
        self.faces = np.stack([ufkey // (Nn * Nn), (ufkey // Nn) % Nn, ufkey % Nn], axis=1)
        self.tet_faces = finv.reshape(Nt, 4)
        self.Nf = self.faces.shape[0]

        # neighbours across faces (-1 = boundary)
        flat_t = np.repeat(np.arange(Nt), 4)
        flat_f = self.tet_faces.ravel()
        order = np.argsort(flat_f, kind="stable")
        counts = np.bincount(flat_f, minlength=self.Nf)
        if counts.max() > 2:
            raise ValueError("non-manifold mesh: a face is shared by more than two tets")
        self.face_count = counts
        starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
        first_t = flat_t[order[starts]]
        second_t = np.where(counts == 2, flat_t[order[np.minimum(starts + 1, len(order) - 1)]], -1)
        other = np.where(flat_t == first_t[flat_f], second_t[flat_f], first_t[flat_f])
        other = np.where(counts[flat_f] == 2, other, -1)
        self.tet_nbr = other.reshape(Nt, 4)

        # boundary sets: faces with one tet, their edges and nodes
        self.wall_face = counts == 1
        wf = self.faces[self.wall_face]
        self.wall_node = np.zeros(Nn, dtype=bool)
        self.wall_node[wf.ravel()] = True
        wall_pairs = np.concatenate([wf[:, [0, 1]], wf[:, [0, 2]], wf[:, [1, 2]]])
        self.wall_edge = np.zeros(self.Ne, dtype=bool)
        self.wall_edge[self.edge_index(wall_pairs)] = True

        # tet orientation
        P = self.xyz[T]
        det = np.einsum("ti,ti->t", P[:, 1] - P[:, 0],
                        np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))
        self.tet_sign = np.sign(det).astype(np.int64)

        self.G = self._grad()
        self.C = self._curl()
        self.D = self._div()

    def edge_index(self, pairs: np.ndarray) -> np.ndarray:
        p = np.sort(np.asarray(pairs, dtype=np.int64), axis=1)
        key = p[:, 0] * self.Nn + p[:, 1]
        ekey = self.edges[:, 0] * self.Nn + self.edges[:, 1]
        idx = np.searchsorted(ekey, key)
        assert np.all(ekey[idx] == key)
        return idx

    def face_index(self, tris: np.ndarray) -> np.ndarray:
        t = np.sort(np.asarray(tris, dtype=np.int64), axis=1)
        Nn = self.Nn
        key = (t[:, 0] * Nn + t[:, 1]) * Nn + t[:, 2]
        fkey = (self.faces[:, 0] * Nn + self.faces[:, 1]) * Nn + self.faces[:, 2]
        idx = np.searchsorted(fkey, key)
        assert np.all(fkey[idx] == key)
        return idx

    def _grad(self):
        Ne = self.Ne
        rows = np.repeat(np.arange(Ne), 2)
        cols = self.edges.ravel()
        vals = np.tile([-1, 1], Ne)
        return sp.csr_matrix((vals, (rows, cols)), shape=(Ne, self.Nn), dtype=np.int64)

    def _curl(self):
        f = self.faces
        ab = self.edge_index(f[:, [0, 1]])
        ac = self.edge_index(f[:, [0, 2]])
        bc = self.edge_index(f[:, [1, 2]])
        Nf = self.Nf
        rows = np.repeat(np.arange(Nf), 3)
        cols = np.stack([bc, ac, ab], axis=1).ravel()
        vals = np.tile([1, -1, 1], Nf)
        return sp.csr_matrix((vals, (rows, cols)), shape=(Nf, self.Ne), dtype=np.int64)

    def _div(self):
        Nt = self.Nt
        rows = np.repeat(np.arange(Nt), 4)
        cols = self.tet_faces.ravel()
        vals = (self.tet_sign[:, None] * np.array([1, -1, 1, -1])[None, :]).ravel()
        return sp.csr_matrix((vals, (rows, cols)), shape=(Nt, self.Nf), dtype=np.int64)

    # interior index sets (PEC walls: wall edges carry e = 0, wall nodes are grounded)
    @property
    def int_edges(self) -> np.ndarray:
        return np.arange(self.Ne) if self.neumann else np.flatnonzero(~self.wall_edge)

    @property
    def int_nodes(self) -> np.ndarray:
        return np.arange(self.Nn) if self.neumann else np.flatnonzero(~self.wall_node)

    def edge_lengths(self) -> np.ndarray:
        d = self.xyz[self.edges[:, 1]] - self.xyz[self.edges[:, 0]]
        return np.sqrt(np.einsum("ei,ei->e", d, d))
