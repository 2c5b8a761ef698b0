"""Mesh preprocessing specification (oracle; test infrastructure only).

The paper fixes none of this (it ships no code and names no ordering); the
readings below make "bit-exact" meaningful by removing every tie:

* Reverse Cuthill-McKee (Cuthill & McKee 1969; George 1971) on the node
  graph i ~ j iff i and j share an element.  Each component starts at the
  unvisited node of minimum degree (ties: smallest original id); a dequeued
  node appends its unvisited neighbours sorted by (degree, original id);
  the final order is reversed.  new_id[old] = position in that order.
* Node blocks (the default numbering; RCM alone is the other choice): given
  bn nodes per owner block and k blocks per band -- both performance
  parameters that the device library chooses and reports, not part of the
  method -- the RCM order is cut into bands of k * bn consecutive
  positions and each band into blocks of bn nodes by recursive coordinate
  bisection, so that a block is a compact patch instead of a sliver of one
  RCM level.  A set S of more than bn nodes is split along the axis of
  largest extent max - min over S (smallest axis on ties), ordered by
  (coordinate, RCM position): the first bn * floor(ceil(|S| / bn) / 2)
  nodes go first, each part recursively; a set of at most bn nodes is one
  block, in RCM order.  new_id[old] = position in the concatenated blocks.
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


def cuthill_mckee(conn, n_nodes):
    """Cuthill-McKee visiting order (list of old ids) and the number of
    breadth-first levels, summed over the components."""
    ptr, nbr = node_adjacency(conn, n_nodes)
    deg = np.diff(ptr)
    starts = np.lexsort((np.arange(n_nodes), deg))   # by (degree, id)
    visited = np.zeros(n_nodes, dtype=bool)
    level = np.zeros(n_nodes, dtype=np.int64)
    order = []
    n_levels = 0
    si = 0
    while len(order) < n_nodes:
        while visited[starts[si]]:
            si += 1
        s = int(starts[si])
        visited[s] = True
        q = deque([s])
        depth = 0
        while q:
            v = q.popleft()
            order.append(v)
            depth = max(depth, int(level[v]))
            nb = nbr[ptr[v]:ptr[v + 1]]
            nb = nb[~visited[nb]]
            if nb.size:
                nb = nb[np.lexsort((nb, deg[nb]))]
                visited[nb] = True
                level[nb] = level[v] + 1
                q.extend(nb.tolist())
        n_levels += depth + 1
    return order, n_levels


def rcm(conn, n_nodes):
    """Reverse Cuthill-McKee; returns new_id (old -> new), int32."""
    order, _ = cuthill_mckee(conn, n_nodes)
    order = np.array(order[::-1], dtype=np.int64)
    new_id = np.empty(n_nodes, dtype=np.int32)
    new_id[order] = np.arange(n_nodes, dtype=np.int32)
    return new_id


def bisect_blocks(nodes, coords, pos, bn):
    """Recursive coordinate bisection of ``nodes`` into blocks of bn nodes
    (module docstring); returns the nodes in block order."""
    nodes = np.asarray(nodes, dtype=np.int64)
    if nodes.size <= bn:
        return nodes[np.argsort(pos[nodes], kind="stable")]
    x = coords[nodes]
    ext = x.max(axis=0) - x.min(axis=0)
    ax = int(np.argmax(ext))                 # first maximum: smallest axis
    o = np.lexsort((pos[nodes], x[:, ax]))
    parts = -(-nodes.size // bn)
    left = bn * (parts // 2)
    return np.concatenate([bisect_blocks(nodes[o[:left]], coords, pos, bn),
                           bisect_blocks(nodes[o[left:]], coords, pos, bn)])


def block_numbering(conn, coords, n_nodes, bn, band_blocks):
    """Node-block numbering (module docstring) with bn nodes per block and
    band_blocks blocks per band; new_id (old -> new), int32."""
    if bn < 1 or band_blocks < 1:
        raise ValueError("bn and band_blocks must be positive")
    order, _ = cuthill_mckee(conn, n_nodes)
    rcm_order = np.array(order[::-1], dtype=np.int64)
    pos = np.empty(n_nodes, dtype=np.int64)
    pos[rcm_order] = np.arange(n_nodes)
    coords = np.asarray(coords, dtype=np.float64)
    band = band_blocks * bn
    out = [bisect_blocks(rcm_order[b0:b0 + band], coords, pos, bn)
           for b0 in range(0, n_nodes, band)]
    seq = np.concatenate(out)
    new_id = np.empty(n_nodes, dtype=np.int32)
    new_id[seq] = np.arange(n_nodes, dtype=np.int32)
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


def preprocess(prob, block_nodes=0, band_blocks=0, order="blocks"):
    """All bit-exact preprocessing results for a problem, as a dict.
    order: "blocks" (node blocks cut from RCM bands: block_nodes nodes per
    block, band_blocks blocks per band, both required) or "rcm" (the
    numbering ignores both)."""
    if order == "rcm":
        new_id = rcm(prob.conn, prob.n_nodes)
    else:
        new_id = block_numbering(prob.conn, prob.coords, prob.n_nodes, block_nodes,
                                 band_blocks)
    eo = element_order(prob.conn, new_id)
    sconn = np.asarray(new_id)[np.asarray(prob.conn)[eo]]
    col = colour_elements(sconn, prob.n_nodes)
    fmap = free_dof_map(prob.n_nodes, prob.dim, prob.dir_nodes, prob.dir_comps)
    return {"perm": new_id, "elem_order": eo, "color": col, "free_index": fmap}


def bandwidth(conn, numbering):
    """max |i - j| over node pairs sharing an element, under ``numbering``."""
    nc = np.asarray(numbering, dtype=np.int64)[np.asarray(conn, dtype=np.int64)]
    return int((nc.max(axis=1) - nc.min(axis=1)).max())
