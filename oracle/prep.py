"""Mesh preprocessing specification (oracle; test infrastructure only).

The paper fixes none of this (it ships no code and names no ordering); the
readings below make "bit-exact" meaningful by removing every tie:

* Reverse Cuthill-McKee (Cuthill & McKee 1969; George 1971) on the node
  graph i ~ j iff i and j share an element.  Each component starts at the
  unvisited node of minimum degree (ties: smallest original id); a dequeued
  node appends its unvisited neighbours sorted by (degree, original id);
  the final order is reversed.  new_id[old] = position in that order.
* Element order: sort by (min new id of the element's nodes, the sorted
  tuple of its new ids, original element index).  Node order inside an
  element is kept.
* Colouring: priority pi(e) = (fmix32(k XOR 0x9E3779B9), k) with k the
  element's position in the sorted order and fmix32 the MurmurHash3 32-bit
  finaliser (public domain, Appleby 2011).  colour(e) is the smallest c >= 0
  not used by any element of higher priority sharing a node with e.
* Free-DOF map: DOF g = node * d + comp in the caller's numbering; free DOFs
  are numbered in increasing g; constrained ones map to -1.
"""
from collections import deque
import numpy as np


def fmix32(h):
    """MurmurHash3 32-bit finaliser (vectorised over uint32 arrays)."""
    h = np.asarray(h, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    m = np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & m
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & m
    h ^= h >> np.uint64(16)
    return h.astype(np.uint32)


def node_adjacency(conn, n_nodes):
    """Sorted neighbour lists of the node graph (i ~ j iff they share an element)."""
    conn = np.asarray(conn, dtype=np.int64)
    k = conn.shape[1]
    a = np.repeat(conn, k, axis=1).reshape(-1)
    b = np.tile(conn, (1, k)).reshape(-1)
    m = a != b
    pairs = np.unique(a[m] * n_nodes + b[m])
    src = pairs // n_nodes
    dst = pairs % n_nodes
    ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.add.at(ptr, src + 1, 1)
    ptr = np.cumsum(ptr)
    return ptr, dst


def rcm(conn, n_nodes):
    """Reverse Cuthill-McKee; returns new_id (old -> new), int32."""
    ptr, nbr = node_adjacency(conn, n_nodes)
    deg = np.diff(ptr)
    starts = np.lexsort((np.arange(n_nodes), deg))   # by (degree, id)
    visited = np.zeros(n_nodes, dtype=bool)
    order = []
    si = 0
    while len(order) < n_nodes:
        while visited[starts[si]]:
            si += 1
        s = int(starts[si])
        visited[s] = True
        q = deque([s])
        while q:
            v = q.popleft()
            order.append(v)
            nb = nbr[ptr[v]:ptr[v + 1]]
            nb = nb[~visited[nb]]
            if nb.size:
                nb = nb[np.lexsort((nb, deg[nb]))]
                visited[nb] = True
                q.extend(nb.tolist())
    order = np.array(order[::-1], dtype=np.int64)
    new_id = np.empty(n_nodes, dtype=np.int32)
    new_id[order] = np.arange(n_nodes, dtype=np.int32)
    return new_id


def element_order(conn, new_id):
    """Permutation of elements (sorted position -> original index), int32."""
    nc = np.asarray(new_id, dtype=np.int64)[np.asarray(conn, dtype=np.int64)]
    srt = np.sort(nc, axis=1)
    keys = [np.arange(conn.shape[0])]
    for c in range(srt.shape[1] - 1, -1, -1):
        keys.append(srt[:, c])
    # lexsort uses the last key as primary: srt[:,0] (= min), then srt[:,1], ...
    return np.lexsort(keys).astype(np.int32)


def colour_elements(sorted_conn, n_nodes):
    """Greedy colouring in decreasing priority (see module docstring).

    sorted_conn: connectivity already in sorted element order, any node
    numbering.  Returns colour per sorted element (int32).
    """
    sorted_conn = np.asarray(sorted_conn, dtype=np.int64)
    ne = sorted_conn.shape[0]
    k = np.arange(ne, dtype=np.int64)
    hsh = fmix32(k ^ 0x9E3779B9).astype(np.int64)
    order = np.lexsort((k, hsh))[::-1]                 # decreasing (hash, k)
    # node -> elements
    flat = sorted_conn.reshape(-1)
    el = np.repeat(k, sorted_conn.shape[1])
    o = np.argsort(flat, kind="stable")
    ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.add.at(ptr, flat + 1, 1)
    ptr = np.cumsum(ptr)
    n2e = el[o]
    colour = np.full(ne, -1, dtype=np.int64)
    conn_l = sorted_conn.tolist()
    ptr_l = ptr.tolist()
    n2e_l = n2e.tolist()
    col_l = colour.tolist()
    for e in order.tolist():
        used = set()
        for n in conn_l[e]:
            for f in n2e_l[ptr_l[n]:ptr_l[n + 1]]:
                c = col_l[f]
                if c >= 0:
                    used.add(c)
        c = 0
        while c in used:
            c += 1
        col_l[e] = c
    return np.array(col_l, dtype=np.int32)


def free_dof_map(n_nodes, dim, dir_nodes, dir_comps):
    """free_index[g] (int32): rank among free DOFs in increasing g, or -1."""
    n_dof = n_nodes * dim
    free = np.ones(n_dof, dtype=bool)
    free[np.asarray(dir_nodes, np.int64) * dim + np.asarray(dir_comps, np.int64)] = False
    out = np.full(n_dof, -1, dtype=np.int32)
    out[free] = np.arange(int(free.sum()), dtype=np.int32)
    return out


def preprocess(prob):
    """All bit-exact preprocessing results for a problem, as a dict."""
    new_id = rcm(prob.conn, prob.n_nodes)
    eo = element_order(prob.conn, new_id)
    sconn = np.asarray(new_id)[np.asarray(prob.conn)[eo]]
    col = colour_elements(sconn, prob.n_nodes)
    fmap = free_dof_map(prob.n_nodes, prob.dim, prob.dir_nodes, prob.dir_comps)
    return {"perm": new_id, "elem_order": eo, "color": col, "free_index": fmap}


def bandwidth(conn, numbering):
    """max |i - j| over node pairs sharing an element, under ``numbering``."""
    nc = np.asarray(numbering, dtype=np.int64)[np.asarray(conn, dtype=np.int64)]
    return int((nc.max(axis=1) - nc.min(axis=1)).max())
