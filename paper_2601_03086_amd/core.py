"""Python view of the C ABI with torch tensors for device memory and streams.

Argument marshalling only: every computation happens in libpfem.so.
"""
import atexit
import ctypes as C
import functools
import weakref

import numpy as np
import torch

from . import _lib as L
from ._lib import check

# Handles still open at interpreter exit are closed here, servers first and
# contexts last, before the HIP runtime itself shuts down.
_LIVE = {k: weakref.WeakSet() for k in ("server", "batch", "mesh", "ctx")}


@atexit.register
def _close_all():
    for kind in ("server", "batch", "mesh", "ctx"):
        for obj in list(_LIVE[kind]):
            try:
                obj.close()
            except Exception:
                pass


def _on_stream(fn):
    """Order a library call after the caller's current torch stream and make
    the caller's stream wait for the library's work before reusing memory."""
    @functools.wraps(fn)
    def wrap(self, *a, **kw):
        ctx = self.ctx
        cur = torch.cuda.current_stream(ctx.device)
        if cur == ctx.stream:        # caller already runs on the library stream
            return fn(self, *a, **kw)
        ctx.stream.wait_stream(cur)
        try:
            # staging copies made by the wrapper run on the library stream too
            with torch.cuda.stream(ctx.stream):
                return fn(self, *a, **kw)
        finally:
            cur.wait_stream(ctx.stream)
    return wrap


MODEL_IDS = {"lin_plane_stress": L.PFEM_LIN_PLANE_STRESS,
             "lin_plane_strain": L.PFEM_LIN_PLANE_STRAIN,
             "lin_3d": L.PFEM_LIN_3D,
             "nh_plane_strain": L.PFEM_NH_PLANE_STRAIN,
             "nh_3d": L.PFEM_NH_3D}
PARAM_IDS = {"E_nu": L.PFEM_PARAM_E_NU, "lame": L.PFEM_PARAM_LAME}
ORDER_IDS = {"blocks": L.PFEM_ORDER_BLOCKS, "rcm": L.PFEM_ORDER_RCM}
ELEM_IDS = {"p1": L.PFEM_ELEM_P1, "q4": L.PFEM_ELEM_Q4, "q8": L.PFEM_ELEM_Q8}
PREC = {"fp64": L.PFEM_FP64, "fp32": L.PFEM_FP32, L.PFEM_FP64: L.PFEM_FP64,
        L.PFEM_FP32: L.PFEM_FP32}
SCATTER = {"owner": L.PFEM_SCATTER_OWNER, "colored": L.PFEM_SCATTER_COLORED,
           "atomic": L.PFEM_SCATTER_ATOMIC}
LAYOUT = {"user": L.PFEM_LAYOUT_USER, "internal": L.PFEM_LAYOUT_INTERNAL}
KRYLOV = {"auto": L.PFEM_KRYLOV_AUTO, "classic": L.PFEM_KRYLOV_CLASSIC,
          "fused": L.PFEM_KRYLOV_FUSED}
PRECOND = {"jacobi": L.PFEM_PRECOND_JACOBI, "two_level": L.PFEM_PRECOND_TWO_LEVEL}


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return C.c_void_p(a.data_ptr())
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    raise TypeError(type(a))


def _dtype(prec):
    return torch.float64 if PREC[prec] == L.PFEM_FP64 else torch.float32


class Context:
    """One device + one HIP stream (a dedicated torch stream by default;
    calls are ordered against the caller's current stream with events)."""

    def __init__(self, device=0, stream=None):
        L.load()
        self.device = torch.device("cuda", device)
        if stream is None:   # a stream of our own (default priority)
            stream = torch.cuda.Stream(device=self.device)
        self.stream = stream
        h = C.c_void_p()
        check(L.pfem_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h
        _LIVE["ctx"].add(self)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            L.pfem_ctx_destroy(self.h)
            self.h = None

    __del__ = close

    def set_timing(self, families=(0, 1, 2, 3, 4, 5, 6), sample_every=1):
        mask = 0
        for f in families or ():
            mask |= 1 << f
        check(L.pfem_ctx_set_timing_sample(self.h, int(sample_every)))
        check(L.pfem_ctx_set_timing(self.h, mask))

    def reset_timing(self):
        check(L.pfem_ctx_reset_timing(self.h))

    def kernel_time(self, family):
        n = C.c_int64()
        ms = C.c_double()
        check(L.pfem_ctx_kernel_time(self.h, family, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def kernel_stats(self, family):
        """pfem_ctx_kernel_stats: launches timed, ms, launches run and
        algorithmic bytes of one family since the last reset."""
        k = L.pfem_kernel_stats()
        check(L.pfem_ctx_kernel_stats(self.h, family, C.byref(k)))
        return {f: getattr(k, f) for f, _ in k._fields_}

    def synchronize(self):
        check(L.pfem_ctx_synchronize(self.h))


class Mesh:
    """A finalized mesh with material and boundary sets (see pfem_mesh_*)."""

    def __init__(self, ctx, dim, coords, conn, model, param_kind, p0, p1,
                 dir_nodes=(), dir_comps=(), dir_values=(), facets=None,
                 traction=None, block_nodes=0, order="blocks", pairs=None, pair_k=0.0,
                 elem="p1"):
        L.load()
        self.ctx = ctx
        self.dim = int(dim)
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.n_nodes = coords.shape[0]
        self.n_elems = conn.shape[0]
        self.n_dof = self.n_nodes * self.dim
        self.model = model
        self.nonlinear = model.startswith("nh")
        self.elem = elem
        h = C.c_void_p()
        if elem == "p1":
            check(L.pfem_mesh_create(ctx.h if ctx is not None else None, self.dim,
                                     self.n_nodes, _ptr(coords), self.n_elems, _ptr(conn),
                                     C.byref(h)))
        else:
            check(L.pfem_mesh_create_quad(ctx.h if ctx is not None else None, ELEM_IDS[elem],
                                          self.n_nodes, _ptr(coords), self.n_elems,
                                          _ptr(conn), C.byref(h)))
        self.h = h
        p0 = np.ascontiguousarray(np.broadcast_to(p0, (self.n_elems,)), dtype=np.float64)
        p1 = np.ascontiguousarray(np.broadcast_to(p1, (self.n_elems,)), dtype=np.float64)
        check(L.pfem_mesh_set_material(h, MODEL_IDS[model], PARAM_IDS[param_kind],
                                       _ptr(p0), _ptr(p1)))
        dn = np.ascontiguousarray(dir_nodes, dtype=np.int32)
        dc = np.ascontiguousarray(dir_comps, dtype=np.int8)
        dv = np.ascontiguousarray(dir_values, dtype=np.float64)
        check(L.pfem_mesh_set_dirichlet(h, dn.size, _ptr(dn), _ptr(dc), _ptr(dv)))
        if facets is not None and len(facets):
            fa = np.ascontiguousarray(facets, dtype=np.int32)
            tr = np.ascontiguousarray(traction, dtype=np.float64)
            check(L.pfem_mesh_set_neumann(h, fa.shape[0], _ptr(fa), _ptr(tr)))
        if pairs is not None and len(pairs):
            pa = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
            check(L.pfem_mesh_set_periodic(h, pa.shape[0], _ptr(pa), float(pair_k)))
        self.periodic = pairs is not None and len(pairs) > 0
        check(L.pfem_mesh_set_node_order(h, ORDER_IDS[order]))
        check(L.pfem_mesh_finalize(h, int(block_nodes)))
        self.info = self.get_info()
        _LIVE["mesh"].add(self)

    @classmethod
    def from_cell(cls, ctx, cell, block_nodes=0, order="blocks"):
        """A periodic cell (homogenisation): linear 3D elements with their
        (E, nu), the periodic springs, and the pin held at zero."""
        pin = np.full(3, cell.pin, dtype=np.int32)
        return cls(ctx, 3, cell.coords, cell.conn, "lin_3d", "E_nu", cell.p0, cell.p1,
                   pin, np.arange(3, dtype=np.int8), np.zeros(3), None, None,
                   block_nodes, order, pairs=cell.pairs, pair_k=cell.penalty)

    @classmethod
    def from_problem(cls, ctx, prob, block_nodes=0, order="blocks"):
        """Build from any object with the fields of a problem description.
        order: internal node numbering, "blocks" (default) or "rcm"."""
        return cls(ctx, prob.coords.shape[1], prob.coords, prob.conn, prob.model,
                   prob.param_kind, prob.p0, prob.p1, prob.dir_nodes, prob.dir_comps,
                   prob.dir_values, prob.neu_facets, prob.neu_traction, block_nodes,
                   order, elem=getattr(prob, "elem", "p1"))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            L.pfem_mesh_destroy(self.h)
            self.h = None

    __del__ = close

    def footprint(self, prec="fp32"):
        """Device bytes of the mesh arrays plus one solve in prec."""
        b = C.c_int64()
        check(L.pfem_mesh_footprint(self.h, PREC[prec], C.byref(b)))
        return b.value

    def prepare_coarse(self):
        """Build the two-level preconditioner's coarse space now (host);
        returns the coarse dimension."""
        n = C.c_int32()
        check(L.pfem_mesh_prepare_coarse(self.h, C.byref(n)))
        return n.value

    def upload(self, ctx):
        """Make a host-only mesh resident on ctx's device."""
        check(L.pfem_mesh_upload(self.h, ctx.h))
        self.ctx = ctx

    def release_device(self):
        """Free the device arrays; the mesh stays usable on the host."""
        check(L.pfem_mesh_release_device(self.h))

    def get_info(self):
        inf = L.pfem_mesh_info()
        check(L.pfem_mesh_get_info(self.h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def query(self, which):
        n = C.c_int64()
        check(L.pfem_mesh_query_int(self.h, which, None, 0, C.byref(n)))
        out = np.empty(n.value, dtype=np.int32)
        check(L.pfem_mesh_query_int(self.h, which, _ptr(out), n.value, C.byref(n)))
        return out

    # ---------------------------------------------------- device vectors
    def new_vec(self, prec="fp64"):
        return torch.empty(self.n_dof, dtype=_dtype(prec), device=self.ctx.device)

    def _vec(self, x, prec):
        t = torch.as_tensor(x, device=self.ctx.device, dtype=_dtype(prec))
        if t.numel() != self.n_dof:
            raise ValueError(f"vector has {t.numel()} entries, mesh has {self.n_dof} DOFs")
        return t.contiguous()

    def _out(self, out, prec):
        """Output vector: a new one, or the caller's, which must be a
        contiguous tensor of n_dof entries of prec's dtype on the context's
        device (the kernels write every entry)."""
        if out is None:
            return self.new_vec(prec)
        if not (isinstance(out, torch.Tensor) and out.device == self.ctx.device
                and out.dtype == _dtype(prec) and out.numel() == self.n_dof
                and out.is_contiguous()):
            raise ValueError(f"out must be a contiguous {_dtype(prec)} tensor of "
                             f"{self.n_dof} entries on {self.ctx.device}")
        return out

    def _host(self, x):
        """Host float64 vector of n_dof entries (the library copies n_dof)."""
        a = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        if a.size != self.n_dof:
            raise ValueError(f"vector has {a.size} entries, mesh has {self.n_dof} DOFs")
        return a

    @_on_stream
    def permute(self, x, to_internal=True, prec="fp64"):
        x = self._vec(x, prec)
        y = torch.empty_like(x)
        check(L.pfem_permute(self.h, PREC[prec], 1 if to_internal else 0, _ptr(x), _ptr(y)))
        return y

    @_on_stream
    def hvp(self, u, v, prec="fp32", layout="user", scatter="owner", mask=0, out=None):
        v = self._vec(v, prec)
        u = self._vec(u, prec) if u is not None else None
        y = self._out(out, prec)
        check(L.pfem_hvp(self.h, PREC[prec], LAYOUT[layout], SCATTER[scatter], mask,
                         _ptr(u), _ptr(v), _ptr(y)))
        return y

    @_on_stream
    def apply_K(self, v, prec="fp32", layout="user", scatter="owner", mask=0, out=None):
        v = self._vec(v, prec)
        y = self._out(out, prec)
        check(L.pfem_apply_K(self.h, PREC[prec], LAYOUT[layout], SCATTER[scatter], mask,
                             _ptr(v), _ptr(y)))
        return y

    @_on_stream
    def force(self, u, prec="fp64", layout="user", mask=0, out=None):
        u = self._vec(u, prec)
        y = self._out(out, prec)
        check(L.pfem_force(self.h, PREC[prec], LAYOUT[layout], mask, _ptr(u), _ptr(y)))
        return y

    @_on_stream
    def energy(self, u, prec="fp64", layout="user"):
        u = self._vec(u, prec)
        e = torch.empty((), dtype=torch.float64, device=self.ctx.device)
        check(L.pfem_energy(self.h, PREC[prec], LAYOUT[layout], _ptr(u), _ptr(e)))
        return e

    @_on_stream
    def energy_noalloc(self, u, prec="fp64", layout="user", out=None):
        """pfem_energy_noalloc: the energy with no allocation inside the
        library (out: an existing float64 device scalar, written in place)."""
        u = self._vec(u, prec)
        e = out if out is not None else torch.empty((), dtype=torch.float64,
                                                    device=self.ctx.device)
        if not (isinstance(e, torch.Tensor) and e.dtype == torch.float64
                and e.device == self.ctx.device and e.numel() == 1):
            raise ValueError("out must be one float64 entry on the context's device")
        check(L.pfem_energy_noalloc(self.h, PREC[prec], LAYOUT[layout], _ptr(u), _ptr(e)))
        return e

    @_on_stream
    def diag(self, u=None, prec="fp64", layout="user"):
        uu = self._vec(u, prec) if u is not None else None
        y = self.new_vec(prec)
        check(L.pfem_diag(self.h, PREC[prec], LAYOUT[layout], _ptr(uu), _ptr(y)))
        return y

    # ------------------------------------------------------------ solve
    @staticmethod
    def opts(tol=1e-8, prec="fp32", tol_fine=0.0, max_iter=0, n_load_steps=10,
             max_newton=50, record_history=1, inner_rtol=0.0, krylov="auto",
             precond="jacobi"):
        o = L.pfem_solve_opts()
        L.pfem_solve_opts_default(C.byref(o))
        o.tol = tol
        o.tol_fine = tol_fine
        o.max_iter = max_iter
        o.n_load_steps = n_load_steps
        o.max_newton = max_newton
        o.prec = PREC[prec]
        o.record_history = record_history
        o.inner_rtol = inner_rtol
        o.krylov = KRYLOV[krylov]
        o.precond = PRECOND[precond]
        return o

    @_on_stream
    def solve(self, u0=None, history_cap=100000, device_io=False, out=None, **kw):
        """Warm-started solve; returns (u, report dict, history ndarray)."""
        o = self.opts(**kw)
        rep = L.pfem_solve_report()
        hist = np.zeros(max(history_cap, 1), dtype=np.float64)
        if device_io:
            u0t = self._vec(u0, "fp64") if u0 is not None else None
            u = self._out(out, "fp64")
            st = L.pfem_solve(self.h, _ptr(u0t), C.byref(o), _ptr(u), 1, _ptr(hist),
                              history_cap, C.byref(rep))
        else:
            u0a = self._host(u0) if u0 is not None else None
            u = np.zeros(self.n_dof, dtype=np.float64)
            st = L.pfem_solve(self.h, _ptr(u0a), C.byref(o), _ptr(u), 0, _ptr(hist),
                              history_cap, C.byref(rep))
        r = rep.as_dict()
        r["status_name"] = L.STATUS_NAMES.get(rep.status, rep.status)
        if st < 0:
            try:
                check(st)
            except L.PfemError as e:   # keep what the failed solve reported
                e.report, e.u, e.history = r, u, hist[:rep.history_len].copy()
                raise
        return u, r, hist[:rep.history_len].copy()


def homogenize(mesh, u0=None, device_io=False, **kw):
    """pfem_homogenize on a periodic cell mesh: returns (fluctuations
    (6, n_dof), E^H (6, 6), list of six report dicts)."""
    o = Mesh.opts(**kw)
    reps = (L.pfem_solve_report * 6)()
    eh = np.zeros(36, dtype=np.float64)
    nd = mesh.n_dof
    ctx = mesh.ctx
    if device_io:
        u0t = None
        if u0 is not None:
            u0t = torch.as_tensor(u0, dtype=torch.float64, device=ctx.device).reshape(-1)
            if u0t.numel() != 6 * nd:
                raise ValueError("u0 must hold 6 n_dof entries")
            u0t = u0t.contiguous()
        x = torch.empty(6 * nd, dtype=torch.float64, device=ctx.device)
        cur = torch.cuda.current_stream(ctx.device)
        ctx.stream.wait_stream(cur)
        st = L.pfem_homogenize(mesh.h, _ptr(u0t), C.byref(o), _ptr(x), 1, _ptr(eh), reps)
        cur.wait_stream(ctx.stream)
        x = x.reshape(6, nd)
    else:
        u0a = None
        if u0 is not None:
            u0a = np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)
            if u0a.size != 6 * nd:
                raise ValueError("u0 must hold 6 n_dof entries")
        x = np.zeros(6 * nd, dtype=np.float64)
        st = L.pfem_homogenize(mesh.h, _ptr(u0a), C.byref(o), _ptr(x), 0, _ptr(eh), reps)
        x = x.reshape(6, nd)
    out = []
    for r in reps:
        d = r.as_dict()
        d["status_name"] = L.STATUS_NAMES.get(r.status, r.status)
        out.append(d)
    if st < 0:
        check(st)
    return x, eh.reshape(6, 6), out


class Batch:
    """Several meshes evaluated by one launch per kernel (internal layout)."""

    def __init__(self, ctx, meshes):
        self.ctx = ctx
        self.meshes = list(meshes)
        arr = (C.c_void_p * len(self.meshes))(*[m.h.value for m in self.meshes])
        h = C.c_void_p()
        check(L.pfem_batch_create(ctx.h, len(self.meshes), arr, C.byref(h)))
        self.h = h
        off = np.zeros(len(self.meshes) + 1, dtype=np.int64)
        check(L.pfem_batch_offsets(h, _ptr(off)))
        self.offsets = off
        self.n_dof = int(off[-1])
        _LIVE["batch"].add(self)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            L.pfem_batch_destroy(self.h)
            self.h = None

    __del__ = close

    def _vec(self, x, prec):
        t = torch.as_tensor(x, device=self.ctx.device, dtype=_dtype(prec))
        if t.numel() != self.n_dof:
            raise ValueError(f"vector has {t.numel()} entries, batch has {self.n_dof} DOFs")
        return t.contiguous()

    @_on_stream
    def energy(self, u, prec="fp32"):
        u = self._vec(u, prec)
        e = torch.empty(len(self.meshes), dtype=torch.float64, device=self.ctx.device)
        check(L.pfem_batch_energy(self.h, PREC[prec], _ptr(u), _ptr(e)))
        return e

    @_on_stream
    def force(self, u, prec="fp32", mask=0):
        u = self._vec(u, prec)
        g = torch.empty_like(u)
        check(L.pfem_batch_force(self.h, PREC[prec], mask, _ptr(u), _ptr(g)))
        return g

    @_on_stream
    def hvp(self, u, v, prec="fp32", mask=0):
        """u may be None when every mesh of the batch is linear."""
        v = self._vec(v, prec)
        u = self._vec(u, prec) if u is not None else None
        y = torch.empty_like(v)
        check(L.pfem_batch_hvp(self.h, PREC[prec], mask, _ptr(u), _ptr(v), _ptr(y)))
        return y


class Server:
    """Continuous-batching solve server (pfem_server_*)."""

    def __init__(self, ctx, hbm_budget_bytes, max_slots=32):
        self.ctx = ctx
        h = C.c_void_p()
        check(L.pfem_server_create(ctx.h, int(hbm_budget_bytes), int(max_slots), C.byref(h)))
        self.h = h
        self._meshes = {}
        _LIVE["server"].add(self)

    def submit(self, req_id, mesh, u0=None, **kw):
        o = Mesh.opts(**kw)
        u0a = mesh._host(u0) if u0 is not None else None
        check(L.pfem_server_submit(self.h, mesh.h, _ptr(u0a), C.byref(o), int(req_id)))
        self._meshes[req_id] = mesh

    def poll(self, cap=1024):
        ids = np.zeros(cap, dtype=np.int64)
        n = C.c_int64()
        check(L.pfem_server_poll(self.h, _ptr(ids), cap, C.byref(n)))
        return ids[:n.value].tolist()

    def result(self, req_id):
        """Collect a finished request (raises PfemError with PFEM_E_STATE
        while it is queued or live; the mesh stays referenced until then)."""
        mesh = self._meshes[req_id]
        u = np.zeros(mesh.n_dof, dtype=np.float64)
        rep = L.pfem_solve_report()
        ts, ta, td = C.c_double(), C.c_double(), C.c_double()
        st = L.pfem_server_result(self.h, int(req_id), _ptr(u), C.byref(rep), C.byref(ts),
                                  C.byref(ta), C.byref(td))
        if st == L.PFEM_E_STATE:
            check(st)
        del self._meshes[req_id]     # released by the library
        r = rep.as_dict()
        r["status_name"] = L.STATUS_NAMES.get(rep.status, rep.status)
        r.update(t_submit=ts.value, t_admit=ta.value, t_done=td.value, call_status=st)
        return u, r

    def cancel(self, req_id):
        check(L.pfem_server_cancel(self.h, int(req_id)))

    def set_timing(self, families=()):
        mask = 0
        for f in families or ():
            mask |= 1 << f
        check(L.pfem_server_set_timing(self.h, mask))

    def kernel_stats(self, family):
        k = L.pfem_kernel_stats()
        check(L.pfem_server_kernel_stats(self.h, family, C.byref(k)))
        return {f: getattr(k, f) for f, _ in k._fields_}

    def stats(self):
        s = L.pfem_server_stats()
        check(L.pfem_server_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in s._fields_}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            L.pfem_server_destroy(self.h)
            self.h = None

    __del__ = close
