"""C-ABI checks that need no GPU: the library loads and exports every symbol
the header declares, and the host-side preprocessing (node numbering,
element order, colouring, free-DOF map, owner blocks) equals the oracle's
bit for bit."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import prep
from tests import meshkit as mk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfem.h")


def _lib():
    from paper_2601_03086_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libpfem.so not built (run __graft_entry__.build())")
    return L


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pfem_[A-Za-z_0-9]+)\s*\(", txt)))


def test_header_symbols_exported():
    L = _lib()
    lib = C.CDLL(L.LIB_PATH)
    names = _declared()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), f"{n} declared in pfem.h but not exported"
    assert sorted(L.PROTOTYPES) == names, "binding prototypes differ from the header"


def test_version_and_error_string():
    L = _lib()
    L.load()
    assert b"gfx950" in L.pfem_version()
    # a call with a NULL handle reports an error without a device
    st = L.pfem_mesh_finalize(None, 0)
    assert st == L.PFEM_E_INVALID_ARG
    assert b"NULL" in L.pfem_last_error()


def _host_mesh(prob, block_nodes=0):
    from paper_2601_03086_amd import core
    return core.Mesh.from_problem(None, prob, block_nodes)


PROBLEMS = {
    "c1": lambda: synth.unit_square_c1(),
    "plate": lambda: synth.plate_problem(31, 32, 33, n_holes=4, target_tris=4000),
    "box": lambda: synth.box_problem(41, 42, n_per_unit=5, n_voids=3, n_load_steps=2),
    "beam_q4": lambda: synth.beam_problem(43, 24, 12),
    "cook_q8": lambda: synth.cook_problem(44, 14),
}


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("order,bn", [("blocks", 0), ("blocks", 32), ("blocks", 96),
                                      ("rcm", 0), ("rcm", 64)])
def test_preprocessing_bit_exact(name, order, bn):
    L = _lib()
    from paper_2601_03086_amd import core
    p = PROBLEMS[name]()
    m = core.Mesh.from_problem(None, p, bn, order)
    # block size and band length are the library's performance choices (the
    # oracle specifies the numbering for given values): read them back
    info = m.info
    if bn:
        assert info["block_nodes"] == bn
    if order == "rcm":
        assert info["band_blocks"] == 0
    else:
        # bands stay within 32768 positions (16-bit packed node offsets)
        assert info["band_blocks"] >= 1
        assert info["band_blocks"] * info["block_nodes"] <= 32768
    ref = prep.preprocess(p, info["block_nodes"], info["band_blocks"], order)
    assert np.array_equal(m.query(L.PFEM_Q_PERM), ref["perm"])
    assert np.array_equal(m.query(L.PFEM_Q_ELEM_ORDER), ref["elem_order"])
    assert np.array_equal(m.query(L.PFEM_Q_COLOR), ref["color"])
    assert np.array_equal(m.query(L.PFEM_Q_FREE_INDEX), ref["free_index"])
    info = m.info
    assert info["n_colors"] == int(ref["color"].max()) + 1
    assert info["bandwidth_internal"] == prep.bandwidth(p.conn, ref["perm"])
    assert info["n_free"] == int((ref["free_index"] >= 0).sum())


@pytest.mark.parametrize("bn", [32, 64, 96])
def test_owner_blocks_cover_every_touch(bn):
    """Each node block's element range contains every element touching it,
    and the owned ranges partition the sorted elements."""
    L = _lib()
    p = synth.plate_problem(51, 52, 53, n_holes=2, target_tris=2500)
    m = _host_mesh(p, block_nodes=bn)
    ref = prep.preprocess(p, bn, m.info["band_blocks"])
    sconn = ref["perm"][p.conn[ref["elem_order"]]]
    blk = m.query(L.PFEM_Q_BLOCKS).reshape(-1, 3)
    nb = (p.n_nodes + bn - 1) // bn
    assert blk.shape[0] == nb == m.info["n_blocks"]
    assert blk[0, 1] == 0 and blk[-1, 2] == p.n_elems
    assert np.all(blk[1:, 1] == blk[:-1, 2])
    owner = sconn.min(axis=1) // bn
    visits = 0
    for b in range(nb):
        touching = np.nonzero(np.any(sconn // bn == b, axis=1))[0]
        visits += touching.size
        assert touching.min() == blk[b, 0]
        assert touching.max() < blk[b, 2]
        own = np.nonzero(owner == b)[0]
        assert own.size == 0 or (own.min() == blk[b, 1] and own.max() == blk[b, 2] - 1)
    # every element is visited once per block it touches, and no more
    assert m.info["owner_elem_visits"] == visits


def test_invalid_meshes_rejected():
    L = _lib()
    from paper_2601_03086_amd import core
    coords = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.float64)
    good = np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)
    cases = {
        "out of range": np.array([[0, 1, 4], [1, 3, 2]], dtype=np.int32),
        "repeated node": np.array([[0, 1, 1], [1, 3, 2]], dtype=np.int32),
        "orphan node": np.array([[0, 1, 2], [0, 1, 2]], dtype=np.int32),
    }
    for what, conn in cases.items():
        with pytest.raises(L.PfemError) as ei:
            core.Mesh(None, 2, coords, conn, "lin_plane_strain", "E_nu", 1.0, 0.3)
        assert ei.value.status == L.PFEM_E_INVALID_MESH, what
    flat = np.array([[0, 0], [1, 0], [2, 0], [1, 1]], dtype=np.float64)
    with pytest.raises(L.PfemError) as ei:
        core.Mesh(None, 2, flat, np.array([[0, 1, 2], [0, 1, 3]], np.int32),
                  "lin_plane_strain", "E_nu", 1.0, 0.3)
    assert ei.value.status == L.PFEM_E_INVALID_MESH
    with pytest.raises(L.PfemError) as ei:
        core.Mesh(None, 2, coords, good, "lin_plane_strain", "E_nu", 1.0, 0.3,
                  dir_nodes=[0, 0], dir_comps=[0, 0], dir_values=[0.0, 1.0])
    assert ei.value.status == L.PFEM_E_INVALID_ARG
    with pytest.raises(L.PfemError) as ei:
        core.Mesh(None, 2, coords, good, "lin_3d", "E_nu", 1.0, 0.3)
    assert ei.value.status == L.PFEM_E_INVALID_ARG
    m = core.Mesh(None, 2, coords, good, "lin_plane_strain", "E_nu", 1.0, 0.3)
    st = L.pfem_energy(m.h, 0, 0, None, None)
    assert st in (L.PFEM_E_STATE, L.PFEM_E_INVALID_ARG)


def test_host_only_mesh_refuses_device_calls():
    L = _lib()
    p = synth.unit_square_c1(n=5)
    m = _host_mesh(p)
    dummy = C.c_void_p(1)
    st = L.pfem_apply_K(m.h, 0, 0, 0, 0, dummy, dummy)
    assert st == L.PFEM_E_STATE
    assert b"device" in L.pfem_last_error()


def test_node_order_rejects_bad_calls():
    L = _lib()
    import ctypes as C
    coords = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.float64)
    conn = np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)
    h = C.c_void_p()
    assert L.pfem_mesh_create(None, 2, 4, coords.ctypes.data, 2, conn.ctypes.data,
                              C.byref(h)) == 0
    try:
        assert L.pfem_mesh_set_node_order(h, 7) == L.PFEM_E_INVALID_ARG
        assert L.pfem_mesh_set_node_order(h, L.PFEM_ORDER_RCM) == 0
        mu = np.ones(2)
        assert L.pfem_mesh_set_material(h, L.PFEM_LIN_PLANE_STRAIN, L.PFEM_PARAM_LAME,
                                        mu.ctypes.data, mu.ctypes.data) == 0
        assert L.pfem_mesh_finalize(h, 0) == 0
        assert L.pfem_mesh_set_node_order(h, L.PFEM_ORDER_BLOCKS) == L.PFEM_E_STATE
    finally:
        L.pfem_mesh_destroy(h)


def test_block_numbering_cuts_straddling_elements():
    """The default numbering visits far fewer elements twice than RCM blocks
    of the same size on a 2D plate and a 3D box (element work per launch)."""
    from paper_2601_03086_amd import core
    for p, bn, gain in [(synth.plate_problem(61, 62, 63, n_holes=3, target_tris=20000), 64, 0.8),
                        (synth.box_problem(71, 72, n_per_unit=8, n_voids=3), 64, 0.85)]:
        v = {o: core.Mesh.from_problem(None, p, bn, o).info["owner_elem_visits"]
             for o in ("blocks", "rcm")}
        assert v["blocks"] <= gain * v["rcm"], (v, p.name)


def test_mesh_beyond_32bit_offsets_rejected():
    """The element kernels address per-node arrays with 32-bit byte offsets;
    the largest is the FP64 fused-PCG record, 96 bytes per 3D node, so a 3D
    mesh of 2^32 / 96 nodes or more is refused at finalize, before any
    preprocessing (disjoint unit tets, every node used)."""
    L = _lib()
    from paper_2601_03086_amd import core
    n_tet = ((1 << 32) // 96 + 4) // 4          # just past the limit
    n = 4 * n_tet
    coords = np.zeros((n, 3))
    base = np.arange(n_tet, dtype=np.float64) * 2.0
    coords[0::4, 0] = base
    coords[1::4, 0] = base + 1.0
    coords[2::4, 0] = base
    coords[2::4, 1] = 1.0
    coords[3::4, 0] = base
    coords[3::4, 2] = 1.0
    conn = np.arange(n, dtype=np.int32).reshape(-1, 4)
    with pytest.raises(L.PfemError) as ei:
        core.Mesh(None, 3, coords, conn, "lin_3d", "E_nu", 1.0, 0.3)
    assert ei.value.status == L.PFEM_E_INVALID_MESH
    assert "too large" in str(ei.value)


@pytest.mark.parametrize("kind", ["plate", "box"])
def test_parallel_colouring_bit_exact(kind):
    """Meshes above the size where the library colours in parallel rounds
    (Jones-Plassmann, several host threads): the colours still equal the
    oracle's sequential greedy in priority order."""
    L = _lib()
    from paper_2601_03086_amd import core
    if kind == "plate":
        p = synth.plate_problem(5, 6, 7, n_holes=3, target_tris=80000)
    else:
        p = synth.box_problem(8, 9, n_per_unit=16, n_voids=3)
    assert p.n_elems >= 65536
    m = core.Mesh.from_problem(None, p)
    col = m.query(L.PFEM_Q_COLOR)
    eo = m.query(L.PFEM_Q_ELEM_ORDER)
    perm = m.query(L.PFEM_Q_PERM)
    sconn = perm[p.conn[eo]]
    assert np.array_equal(col, prep.colour_elements(sconn, p.n_nodes))


def test_colouring_high_degree_node_bit_exact():
    """A 5000-triangle fan (every element shares the centre node, so all
    need distinct colours): the library's colours -- its rounds finish with
    the sequential greedy, using per-node colour sets at nodes of very high
    degree -- equal the oracle's greedy in priority order."""
    L = _lib()
    from paper_2601_03086_amd import core
    from tests import meshkit as mk
    p = mk.fan_problem(m=5000)
    m = core.Mesh.from_problem(None, p, 0, "rcm")
    col = m.query(L.PFEM_Q_COLOR)
    perm = m.query(L.PFEM_Q_PERM)
    sconn = perm[p.conn[m.query(L.PFEM_Q_ELEM_ORDER)]]
    assert m.info["n_colors"] == 5000
    assert np.array_equal(col, prep.colour_elements(sconn, p.n_nodes))


def test_every_entry_point_rejects_null_arguments():
    """Every status-returning call reports PFEM_E_INVALID_ARG when its
    handles and pointers are NULL (no device is touched, nothing crashes),
    and the void destructors accept NULL."""
    L = _lib()
    lib = L.load()
    ints = (C.c_int, L._I32, L._I64, L._D)
    for name, (res, args) in L.PROTOTYPES.items():
        if not args:
            continue
        st = getattr(lib, name)(*[0 if a in ints else None for a in args])
        if res is None:
            assert st is None, name
        else:
            assert st == L.PFEM_E_INVALID_ARG, (name, st)
            assert L.pfem_last_error(), name
    # a NULL handle is caught before any other argument is looked at: the
    # other pointers point at valid host memory and the counts are 1
    buf = C.create_string_buffer(1 << 20)
    first_not_handle = {"pfem_ctx_create", "pfem_mesh_create", "pfem_mesh_create_quad",
                        "pfem_last_error",
                        "pfem_version", "pfem_solve_opts_default"}
    for name, (res, args) in L.PROTOTYPES.items():
        if name in first_not_handle or res is None:
            continue
        vals = [None] + [1 if a in ints else C.cast(buf, a) for a in args[1:]]
        st = getattr(lib, name)(*vals)
        assert st == L.PFEM_E_INVALID_ARG, (name, st)


def test_mesh_setters_reject_bad_arguments():
    L = _lib()
    lib = L.load()
    coords = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.float64)
    conn = np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)
    cp, kp = coords.ctypes.data, conn.ctypes.data
    other = C.c_void_p()
    E = L.PFEM_E_INVALID_ARG
    assert lib.pfem_mesh_create(None, 2, 4, None, 2, kp, C.byref(other)) == E
    assert lib.pfem_mesh_create(None, 2, 4, cp, 2, None, C.byref(other)) == E
    assert lib.pfem_mesh_create(None, 4, 4, cp, 2, kp, C.byref(other)) == E
    assert lib.pfem_mesh_create(None, 2, -1, cp, 2, kp, C.byref(other)) == L.PFEM_E_INVALID_MESH
    h = C.c_void_p()
    assert lib.pfem_mesh_create(None, 2, 4, cp, 2, kp, C.byref(h)) == 0
    try:
        p = np.ones(2)
        assert lib.pfem_mesh_set_material(h, L.PFEM_LIN_PLANE_STRAIN, 0, None, None) == E
        assert lib.pfem_mesh_set_material(h, L.PFEM_LIN_PLANE_STRAIN, 0, p.ctypes.data, None) == E
        assert lib.pfem_mesh_set_material(h, 9, 0, p.ctypes.data, p.ctypes.data) == E
        assert lib.pfem_mesh_set_material(h, L.PFEM_LIN_PLANE_STRAIN, 5,
                                          p.ctypes.data, p.ctypes.data) == E
        assert lib.pfem_mesh_set_dirichlet(h, 3, None, None, None) == E
        assert lib.pfem_mesh_set_dirichlet(h, -3, None, None, None) == E
        assert lib.pfem_mesh_set_neumann(h, 3, None, None) == E
        assert lib.pfem_mesh_finalize(h, 0) == L.PFEM_E_STATE      # no material yet
        assert lib.pfem_mesh_finalize(h, -5) == E
    finally:
        lib.pfem_mesh_destroy(h)


def test_host_only_mesh_calls():
    """A mesh created without a context preprocesses on the host; every call
    that needs the device reports PFEM_E_STATE, and the query hook answers
    a length-only request (out NULL) and truncates to cap."""
    L = _lib()
    lib = L.load()
    prob = synth.unit_square_c1(n=5)
    nn = len(prob.coords)
    m = _host_mesh(prob)
    ints = (C.c_int, L._I32, L._I64)
    for name in ("pfem_hvp", "pfem_apply_K", "pfem_force", "pfem_energy",
                 "pfem_diag", "pfem_permute"):
        args = L.PROTOTYPES[name][1]
        st = getattr(lib, name)(m.h, *[0 if a in ints else None for a in args[1:]])
        assert st == L.PFEM_E_STATE, (name, st)
        assert b"device" in L.pfem_last_error(), name
    # the allocation-free energy checks the mesh state before any device call
    dummy = np.zeros(4)
    st = lib.pfem_energy_noalloc(m.h, L.PFEM_FP64, L.PFEM_LAYOUT_USER,
                                 dummy.ctypes.data, dummy.ctypes.data)
    assert st == L.PFEM_E_STATE and b"device" in L.pfem_last_error()
    assert lib.pfem_energy_noalloc(m.h, 7, L.PFEM_LAYOUT_USER, dummy.ctypes.data,
                                   dummy.ctypes.data) == L.PFEM_E_INVALID_ARG
    n = L._I64()
    assert lib.pfem_mesh_query_int(m.h, L.PFEM_Q_PERM, None, 0, C.byref(n)) == 0
    assert n.value == nn
    buf = np.full(8, -7, np.int32)
    assert lib.pfem_mesh_query_int(m.h, L.PFEM_Q_PERM, buf.ctypes.data, 5, None) == 0
    full = np.zeros(nn, np.int32)
    assert lib.pfem_mesh_query_int(m.h, L.PFEM_Q_PERM, full.ctypes.data, nn, C.byref(n)) == 0
    assert np.array_equal(buf[:5], full[:5]) and (buf[5:] == -7).all()
    assert sorted(full.tolist()) == list(range(nn))
    assert lib.pfem_mesh_query_int(m.h, 99, None, 0, None) == L.PFEM_E_INVALID_ARG
    assert lib.pfem_mesh_query_int(m.h, L.PFEM_Q_PERM, full.ctypes.data, -1, None) \
        == L.PFEM_E_INVALID_ARG


def test_solve_options_checked_before_the_device():
    """pfem_solve rejects bad options with PFEM_E_INVALID_ARG before it
    looks for a device; good options on a host-only mesh then give
    PFEM_E_STATE.  An inner reduction of 1 or more would end every
    refinement sweep at iteration 0 and never finish."""
    L = _lib()
    lib = L.load()
    m = _host_mesh(synth.unit_square_c1(n=5))
    u = np.zeros(m.n_dof)

    def solve(**kw):
        o = L.pfem_solve_opts()
        lib.pfem_solve_opts_default(C.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return lib.pfem_solve(m.h, None, C.byref(o), u.ctypes.data, 0, None, 0, None)

    assert solve() == L.PFEM_E_STATE
    assert solve(inner_rtol=0.5) == L.PFEM_E_STATE
    for bad in (dict(tol=0.0), dict(tol=-1.0), dict(tol=float("nan")), dict(tol=float("inf")),
                dict(prec=7), dict(krylov=9), dict(inner_rtol=0.7), dict(inner_rtol=1.0),
                dict(inner_rtol=-1e-3), dict(inner_rtol=float("nan"))):
        assert solve(**bad) == L.PFEM_E_INVALID_ARG, bad
        assert L.pfem_last_error(), bad


@pytest.mark.parametrize("dim,model,kind,p0,p1,ok", [
    (2, "lin_plane_strain", "E_nu", 1.0, 0.3, True),
    (2, "lin_plane_strain", "E_nu", 0.0, 0.3, False),        # mu = 0
    (2, "lin_plane_strain", "E_nu", -2.0, 0.3, False),       # mu < 0
    (2, "nh_plane_strain", "lame", 1.0, -0.9, True),         # lambda + mu > 0
    (2, "nh_plane_strain", "lame", 1.0, -1.1, False),        # lambda + mu < 0
    (2, "lin_plane_stress", "E_nu", 1.0, 0.7, True),         # lambda* + mu > 0
    (3, "lin_3d", "lame", 1.0, -0.6, True),                  # 3 lambda + 2 mu > 0
    (3, "nh_3d", "lame", 1.0, -0.7, False),                  # 3 lambda + 2 mu < 0
    (3, "lin_3d", "lame", 0.0, 1.0, False),
])
def test_material_must_be_positive_definite(dim, model, kind, p0, p1, ok):
    """Element stiffness is SPD iff mu > 0 and dim * lambda + 2 mu > 0; other
    materials are refused when set, and the mesh keeps no material."""
    L = _lib()
    from paper_2601_03086_amd import core
    if dim == 2:
        coords = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.float64)
        conn = np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)
    else:
        coords = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
        conn = np.array([[0, 1, 2, 3]], dtype=np.int32)
    if ok:
        core.Mesh(None, dim, coords, conn, model, kind, p0, p1)
        return
    with pytest.raises(L.PfemError) as ei:
        core.Mesh(None, dim, coords, conn, model, kind, p0, p1)
    assert ei.value.status == L.PFEM_E_INVALID_ARG
    assert "positive definite" in str(ei.value)


def test_binding_checks_vector_sizes():
    """The binding refuses vectors the library would read or write past:
    output tensors of the wrong size, dtype, device or layout, and host
    vectors of the wrong length (the library copies n_dof entries)."""
    import types

    import torch
    from paper_2601_03086_amd import core
    m = _host_mesh(synth.unit_square_c1(n=5))
    m.ctx = types.SimpleNamespace(device=torch.device("cpu"))   # stand-in device
    try:
        n = m.n_dof
        ok = torch.empty(n, dtype=torch.float32)
        assert m._out(ok, "fp32") is ok
        assert m._out(None, "fp64").shape == (n,)
        for bad in (torch.empty(n - 1, dtype=torch.float32),
                    torch.empty(n, dtype=torch.float64),
                    torch.empty(2 * n, dtype=torch.float32)[::2],
                    np.empty(n, np.float32)):
            with pytest.raises(ValueError):
                m._out(bad, "fp32")
        assert m._host(np.arange(n)).dtype == np.float64
        with pytest.raises(ValueError):
            m._host(np.zeros(n - 1))
        with pytest.raises(ValueError):
            m._vec(torch.zeros(n + 2), "fp32")
    finally:
        m.ctx = None


def test_header_is_c_and_host_calls_work_from_c(tmp_path):
    """include/pfem.h compiles as C99 with warnings as errors, and a C
    program linked against the library drives a host-only mesh."""
    import shutil
    import subprocess
    L = _lib()
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    libdir = os.path.dirname(L.LIB_PATH)
    exe = str(tmp_path / "c_abi_host")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror",
                        "-I" + os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "c_abi_host.c"),
                        "-L" + libdir, "-lpfem", "-Wl,-rpath," + libdir, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "c abi ok" in r.stdout, r.stdout + r.stderr


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message
    (before anything touches a device)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_missing_library_fails_loudly(tmp_path):
    """With libpfem.so absent the package raises on load: there is no CPU
    or PyTorch fallback for any step of the path."""
    import subprocess
    import sys
    code = ("import paper_2601_03086_amd._lib as L\n"
            f"L.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
            "L._lib = None\n"
            "try:\n"
            "    L.load()\n"
            "except ImportError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    print('loaded')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert "raised:" in r.stdout and "absent.so" in r.stdout, r.stdout + r.stderr


def test_oracle_and_library_share_no_code():
    """The package (Python and C++/HIP sources) never names the oracle, the
    oracle never names the package, and the shared input generators import
    neither."""
    import glob
    import re
    pkg = os.path.join(ROOT, "paper_2601_03086_amd")
    for f in glob.glob(os.path.join(pkg, "*.py")) + glob.glob(os.path.join(pkg, "csrc", "*")):
        txt = open(f, errors="replace").read()
        assert not re.search(r"\boracle\b", txt), f
    for f in glob.glob(os.path.join(ROOT, "oracle", "*.py")):
        txt = open(f).read()
        assert "paper_2601_03086_amd" not in txt and "libpfem" not in txt, f
    for f in glob.glob(os.path.join(ROOT, "synth", "*.py")):
        txt = open(f).read()
        assert not re.search(r"^\s*(from|import)\s+(oracle|paper_2601_03086_amd)", txt, re.M), f


def test_coarse_aggregates_and_preparation():
    """PFEM_Q_AGGREGATE: groups of consecutive owner blocks, at most 1536
    coarse DOFs; pfem_mesh_prepare_coarse builds the coarse space on the
    host (no device); the two-level option is checked before the device."""
    import synth
    L = _lib()
    from paper_2601_03086_amd import core
    for p, nrb in ((synth.plate_problem(5, 6, 7, n_holes=2, target_tris=4000), 3),
                   (synth.box_problem(8, 9, n_per_unit=5, n_voids=1, n_load_steps=1), 6)):
        m = core.Mesh.from_problem(None, p, 32)
        agg = m.query(L.PFEM_Q_AGGREGATE)
        perm = m.query(L.PFEM_Q_PERM)
        blocks = perm // m.info["block_nodes"]
        G = -(-nrb * m.info["n_blocks"] // 1536)
        assert np.array_equal(agg, blocks // max(G, 1))
        n_c = m.prepare_coarse()
        assert n_c == nrb * (agg.max() + 1) and n_c <= 1536
        assert m.prepare_coarse() == n_c          # built once
    o = core.Mesh.opts(precond="two_level", krylov="fused")
    u = np.zeros(m.n_dof)
    st = L.load().pfem_solve(m.h, None, C.byref(o), u.ctypes.data, 0, None, 0, None)
    assert st == L.PFEM_E_INVALID_ARG
    o = core.Mesh.opts()
    o.precond = 7
    st = L.load().pfem_solve(m.h, None, C.byref(o), u.ctypes.data, 0, None, 0, None)
    assert st == L.PFEM_E_INVALID_ARG


@pytest.mark.parametrize("elem", ["q4", "q8"])
def test_quad_mesh_info_loads_and_refusals(elem):
    """A quadrilateral mesh reports its family, its consistent loads match
    the oracle's (Q8 edges: quadratic shape functions), and the paths that
    do not cover quadrilaterals are refused without a device."""
    from paper_2601_03086_amd import core
    from oracle import fe
    L = _lib()
    p = synth.beam_problem(45, 16, 6, elem=elem) if elem == "q4" else synth.cook_problem(46, 10)
    m = core.Mesh.from_problem(None, p)
    assert m.info["elem"] == (L.PFEM_ELEM_Q4 if elem == "q4" else L.PFEM_ELEM_Q8)
    assert m.info["nodes_per_elem"] == p.conn.shape[1]
    f = fe.Model(p).f_ext
    assert abs(m.info["f_ext_norm"] - np.linalg.norm(f)) <= 1e-14 * np.linalg.norm(f)
    with pytest.raises(L.PfemError) as e:
        m.prepare_coarse()
    assert e.value.status == L.PFEM_E_INVALID_ARG


def test_quad_mesh_validation():
    """Folded and degenerate quadrilaterals and a wrong family are refused."""
    L = _lib()
    L.load()
    import ctypes as C
    coords = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [2, 0], [2, 1]], np.float64)
    good = np.array([[0, 1, 2, 3], [1, 4, 5, 2]], np.int32)
    folded = np.array([[0, 1, 2, 3], [1, 4, 2, 5]], np.int32)    # bow-tie
    flat = np.array([[0, 1, 4, 3]], np.int32)                    # three corners on a line

    def make(conn, elem=L.PFEM_ELEM_Q4):
        h = C.c_void_p()
        st = L.pfem_mesh_create_quad(None, elem, coords.shape[0], coords.ctypes.data,
                                     conn.shape[0], conn.ctypes.data, C.byref(h))
        if st != 0:
            return st, None
        ne = conn.shape[0]
        E, nu = np.full(ne, 1.0), np.full(ne, 0.3)
        assert L.pfem_mesh_set_material(h, L.PFEM_LIN_PLANE_STRAIN, L.PFEM_PARAM_E_NU,
                                        E.ctypes.data, nu.ctypes.data) == 0
        st = L.pfem_mesh_finalize(h, 0)
        L.pfem_mesh_destroy(h)
        return st, h

    assert make(good)[0] == 0
    assert make(folded)[0] == L.PFEM_E_INVALID_MESH
    assert make(flat)[0] in (L.PFEM_E_INVALID_MESH,)
    assert make(good, elem=7)[0] == L.PFEM_E_INVALID_ARG


@pytest.mark.parametrize("kind", ["plate", "box", "beam_q4"])
def test_solve_footprint_counts_the_neo_hookean_element_cache(kind):
    """The footprint a server admits by includes the per-element cache of
    {F^-T, ln J} that a Neo-Hookean solve on P1 elements keeps for each
    Newton step: (d^2 + 1) values per element in the kernel precision,
    and nothing else differs from the linear model on the same mesh
    (quadrilateral meshes keep no cache)."""
    if kind == "plate":
        make = lambda model: synth.plate_problem(51, 52, 53, n_holes=2, target_tris=3000,
                                                 model=model)
        models = ("lin_plane_strain", "nh_plane_strain")
    elif kind == "box":
        make = lambda model: synth.box_problem(54, 55, n_per_unit=5, n_voids=2, model=model,
                                               n_load_steps=1)
        models = ("lin_3d", "nh_3d")
    else:
        make = lambda model: synth.beam_problem(56, 12, 6, model=model)
        models = ("lin_plane_strain", "nh_plane_strain")
    lin, nh = (_host_mesh(make(mo)) for mo in models)
    d, ne = lin.info["dim"], lin.info["n_elems"]
    vals = (d * d + 1) * ne if kind != "beam_q4" else 0
    assert nh.info["solve_bytes_fp32"] - lin.info["solve_bytes_fp32"] == 4 * vals
    assert nh.info["solve_bytes_fp64"] - lin.info["solve_bytes_fp64"] == 8 * vals
    assert nh.footprint("fp32") == nh.info["device_bytes"] + nh.info["solve_bytes_fp32"]
