"""DEC steady diffusion on tetrahedral meshes for MI355X (gfx950).

Thin Python binding over the C ABI of libdec_hip.so (include/dec.h): every
step of the path -- topology, circumcentric Hodge star with cracks,
assembly of L = d0^T *1 d0, boundary data, PCG / mixed-precision
refinement, flux and effective conductivity -- runs in the HIP kernels of
that library.  This module only checks and marshals arguments; PyTorch
provides device memory (its caching allocator backs the library's
allocations) and streams.
"""
import atexit
import ctypes
import os
import weakref

import torch

from . import _lib
from ._lib import (DEC_FMT_AUTO, DEC_FMT_CSR, DEC_FMT_SELL, DEC_NORM_ENERGY, DEC_NORM_RESIDUAL, DEC_PREC_FP64,
                   DEC_PREC_MIXED, DEC_PRECOND_BLOCK, DEC_PRECOND_FSAI, DEC_PRECOND_JACOBI, SolveOpts,
                   SolveStats)

__all__ = ["DecError", "Context", "Mesh", "DualMesh", "read_tetgen", "Server", "SolveOpts", "SolveStats", "DEC_PREC_FP64", "DEC_PREC_MIXED",
           "DEC_PRECOND_JACOBI", "DEC_PRECOND_FSAI", "DEC_FMT_AUTO", "DEC_FMT_CSR", "DEC_FMT_SELL",
           "DEC_NORM_RESIDUAL", "DEC_NORM_ENERGY", "DEC_PRECOND_BLOCK"]


_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    """Release every library object before torch (whose allocator backs them) shuts down."""
    for ctx in list(_LIVE):
        try:
            ctx.close()
        except Exception:
            pass


class DecError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{_lib.STATUS.get(code, code)}: {message}")
        self.code = code


def read_tetgen(node_path, ele_path):
    """TetGen .node / .ele files (dec_tetgen_read, host only): returns numpy arrays xyz [V,3]
    float64, tets [T,4] int32 (0-based) and the node boundary markers [V] int32."""
    import numpy as np

    lib = _lib.load()
    V, T = ctypes.c_int64(), ctypes.c_int64()
    args = (os.fsencode(node_path), os.fsencode(ele_path))
    rc = lib.dec_tetgen_read(*args, ctypes.byref(V), ctypes.byref(T), None, None, None)
    if rc != 0:
        raise DecError(rc, "dec_tetgen_read: " + lib.dec_last_error(None).decode(errors="replace"))
    xyz = np.empty((V.value, 3), dtype=np.float64)
    tets = np.empty((T.value, 4), dtype=np.int32)
    mark = np.empty(V.value, dtype=np.int32)
    rc = lib.dec_tetgen_read(*args, None, None, xyz.ctypes.data_as(ctypes.c_void_p),
                             tets.ctypes.data_as(ctypes.c_void_p), mark.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise DecError(rc, "dec_tetgen_read: " + lib.dec_last_error(None).decode(errors="replace"))
    return xyz, tets, mark


def _ptr(t, dtype, n=None, name="array"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A dec_ctx bound to a CUDA device and a torch stream; allocations go through torch."""

    def __init__(self, device=None, stream=None, torch_allocator=True):
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        dev_index = self.device.index if self.device.index is not None else 0
        if torch_allocator:
            s = self.stream

            def _alloc(size, user):
                try:
                    return torch.cuda.caching_allocator_alloc(size, dev_index, s)
                except Exception:
                    return None

            def _free(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc = _lib.ALLOC_FN(_alloc)
            self._free = _lib.FREE_FN(_free)
        else:
            self._alloc = ctypes.cast(None, _lib.ALLOC_FN)
            self._free = ctypes.cast(None, _lib.FREE_FN)
        h = ctypes.c_void_p()
        rc = self.lib.dec_create(ctypes.byref(h), dev_index, ctypes.c_void_p(self.stream.cuda_stream),
                                 self._alloc, self._free, None)
        if rc != 0:
            raise DecError(rc, "dec_create failed")
        self.handle = h
        self._children = weakref.WeakSet()  # meshes and servers: closed before the context
        _LIVE.add(self)

    def check(self, rc, what):
        if rc != 0:
            msg = self.lib.dec_last_error(self.handle).decode(errors="replace")
            raise DecError(rc, f"{what}: {msg}")
        return rc

    def close(self):
        if getattr(self, "handle", None):
            for child in list(self._children):
                child.close()
            self.lib.dec_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mesh(self, xyz, tets):
        return Mesh(self, xyz, tets)

    def reorder(self, xyz, tets, order="lexicographic"):
        """Spatial numbering (dec_reorder), order "lexicographic" (the paper's z, y, x) or "morton":
        returns (xyz, tets, vperm, tperm) device tensors, the permutations mapping new to old."""
        code = {"lexicographic": 0, "morton": 1}[order]
        V, T = int(xyz.shape[0]), int(tets.shape[0])
        xo = torch.empty((V, 3), dtype=torch.float64, device=self.device)
        to = torch.empty((T, 4), dtype=torch.int32, device=self.device)
        vp = torch.empty(V, dtype=torch.int32, device=self.device)
        tp = torch.empty(T, dtype=torch.int32, device=self.device)
        rc = self.lib.dec_reorder(self.handle, code, V, _ptr(xyz, torch.float64, 3 * V, "xyz"), T,
                                  _ptr(tets, torch.int32, 4 * T, "tets"), _ptr(xo, torch.float64),
                                  _ptr(to, torch.int32), _ptr(vp, torch.int32), _ptr(tp, torch.int32))
        self.check(rc, "dec_reorder")
        return xo, to, vp, tp


class Mesh:
    """dec_mesh: topology built from (xyz [V,3] float64, tets [T,4] int32) device tensors."""

    def __init__(self, ctx, xyz, tets):
        self.ctx = ctx
        self.lib = ctx.lib
        V, T = int(xyz.shape[0]), int(tets.shape[0])
        h = ctypes.c_void_p()
        rc = self.lib.dec_build_topology(ctx.handle, V, _ptr(xyz, torch.float64, 3 * V, "xyz"), T,
                                         _ptr(tets, torch.int32, 4 * T, "tets"), ctypes.byref(h))
        ctx.check(rc, "dec_build_topology")
        self._adopt(h)

    def _adopt(self, h):
        self.handle = h
        self.ctx._children.add(self)
        vals = [ctypes.c_int64() for _ in range(6)]
        self.ctx.check(self.lib.dec_mesh_info(h, *[ctypes.byref(v) for v in vals]), "dec_mesh_info")
        self.V, self.T, self.E, self.F, self.F_boundary, self.nnz = (v.value for v in vals)

    @property
    def dev(self):
        return self.ctx.device

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dec_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def edges(self):
        out = torch.empty((self.E, 2), dtype=torch.int32, device=self.dev)
        self.ctx.check(self.lib.dec_get_edges(self.handle, _ptr(out, torch.int32)), "dec_get_edges")
        return out

    def csr(self, values=True):
        rp = torch.empty(self.V + 1, dtype=torch.int32, device=self.dev)
        col = torch.empty(self.nnz, dtype=torch.int32, device=self.dev)
        v64 = torch.empty(self.nnz, dtype=torch.float64, device=self.dev) if values else None
        v32 = torch.empty(self.nnz, dtype=torch.float32, device=self.dev) if values else None
        self.ctx.check(self.lib.dec_get_csr(self.handle, _ptr(rp, torch.int32), _ptr(col, torch.int32),
                                            _ptr(v64, torch.float64), _ptr(v32, torch.float32)), "dec_get_csr")
        return rp, col, v64, v32

    def hodge1(self, kappa=None, cracks=None, want_cut=True, want_star=True):
        n = 0 if cracks is None else int(cracks.shape[0])
        cut = torch.empty(self.E, dtype=torch.uint8, device=self.dev) if want_cut else None
        star = torch.empty(self.E, dtype=torch.float64, device=self.dev) if want_star else None
        rc = self.lib.dec_hodge1(self.handle, _ptr(kappa, torch.float64, self.E, "kappa"), n,
                                 _ptr(cracks, torch.float64, 7 * n, "cracks") if n else None,
                                 _ptr(cut, torch.uint8), _ptr(star, torch.float64))
        self.ctx.check(rc, "dec_hodge1")
        return cut, star

    def assemble(self, full_pattern=False):
        """Assemble L; the solver's sliced-ELL copy drops zero-dual-area edges unless full_pattern."""
        self.ctx.check(self.lib.dec_assemble(self.handle, 1 if full_pattern else 0), "dec_assemble")

    def apply_bc(self, bc_type, bc_value, neumann_f0=None, want_rhs=True):
        npin = ctypes.c_int64()
        b = torch.empty(self.V, dtype=torch.float64, device=self.dev) if want_rhs else None
        rc = self.lib.dec_apply_bc(self.handle, _ptr(bc_type, torch.int8, self.V, "bc_type"),
                                   _ptr(bc_value, torch.float64, self.V, "bc_value"),
                                   _ptr(neumann_f0, torch.float64, self.V, "neumann_f0"), ctypes.byref(npin),
                                   _ptr(b, torch.float64))
        self.ctx.check(rc, "dec_apply_bc")
        return npin.value, b

    @staticmethod
    def options(**kw):
        o = SolveOpts()
        _lib.load().dec_solve_opts_default(ctypes.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        return o

    def solve(self, T=None, opts=None, check=True, **kw):
        """Solve the system; returns (T, stats dict, status)."""
        o = opts if opts is not None else self.options(**kw)
        if T is None:
            T = torch.zeros(self.V, dtype=torch.float64, device=self.dev)
        st = SolveStats()
        rc = self.lib.dec_solve(self.handle, ctypes.byref(o), _ptr(T, torch.float64, self.V, "T"), ctypes.byref(st))
        if check:
            self.ctx.check(rc, "dec_solve")
        return T, st.as_dict(), rc

    def solve_noalloc(self, T=None, opts=None, check=True, **kw):
        """dec_solve_noalloc: FP64 Jacobi PCG whose scratch is the library's static device array
        (no allocation inside the call); T (allocated here when None) receives the solution.
        Returns (T, stats dict, status)."""
        o = opts if opts is not None else self.options(**kw)
        if T is None:
            T = torch.zeros(self.V, dtype=torch.float64, device=self.dev)
        st = SolveStats()
        rc = self.lib.dec_solve_noalloc(self.handle, ctypes.byref(o), _ptr(T, torch.float64, self.V, "T"),
                                        ctypes.byref(st))
        if check:
            self.ctx.check(rc, "dec_solve_noalloc")
        return T, st.as_dict(), rc

    def spmv(self, x, y=None, precision=DEC_PREC_FP64, fmt=DEC_FMT_SELL):
        dt = torch.float64 if precision == DEC_PREC_FP64 else torch.float32
        if y is None:
            y = torch.empty(self.V, dtype=dt, device=self.dev)
        self.ctx.check(self.lib.dec_spmv(self.handle, precision, fmt, _ptr(x, dt, self.V, "x"), _ptr(y, dt, self.V, "y")),
                       "dec_spmv")
        return y

    def fsai(self):
        nnz = ctypes.c_int64()
        self.ctx.check(self.lib.dec_get_fsai(self.handle, ctypes.byref(nnz), None, None, None), "dec_get_fsai")
        ptr = torch.empty(self.V + 1, dtype=torch.int32, device=self.dev)
        col = torch.empty(nnz.value, dtype=torch.int32, device=self.dev)
        val = torch.empty(nnz.value, dtype=torch.float64, device=self.dev)
        self.ctx.check(self.lib.dec_get_fsai(self.handle, ctypes.byref(nnz), _ptr(ptr, torch.int32),
                                             _ptr(col, torch.int32), _ptr(val, torch.float64)), "dec_get_fsai")
        return ptr, col, val

    def flux(self, T, side=None, length=1.0, area=1.0, dT=1.0, want_edge_flux=False):
        vals = [ctypes.c_double() for _ in range(4)]
        ef = torch.empty(self.E, dtype=torch.float64, device=self.dev) if want_edge_flux else None
        rc = self.lib.dec_flux_effective_conductivity(
            self.handle, _ptr(T, torch.float64, self.V, "T"), _ptr(side, torch.int8, self.V, "side"),
            length, area, dT, *[ctypes.byref(v) for v in vals], _ptr(ef, torch.float64))
        self.ctx.check(rc, "dec_flux_effective_conductivity")
        k, qi, qo, en = (v.value for v in vals)
        return {"k_eff": k, "q_in": qi, "q_out": qo, "energy": en, "edge_flux": ef}

    def max_flux_edge(self, T, eligible=None):
        """(edge, density) of the face with the largest heat-flux density (-1 when none)."""
        e, d = ctypes.c_int64(), ctypes.c_double()
        rc = self.lib.dec_max_flux_edge(self.handle, _ptr(T, torch.float64, self.V, "T"),
                                        _ptr(eligible, torch.uint8, self.E, "eligible"), ctypes.byref(e),
                                        ctypes.byref(d))
        self.ctx.check(rc, "dec_max_flux_edge")
        return e.value, d.value

    def rms_error(self, T, field=(1.0, -1.0, 0.0, 0.0)):
        """Eq. 15 against the linear field a + g.p, field = (a, gx, gy, gz): T per vertex
        (length V) or per tet (length T, tet systems' solutions)."""
        n = int(T.numel())
        if n not in (self.V, self.T):
            raise ValueError(f"T must have {self.V} (vertex) or {self.T} (tet) values")
        on_tets = 1 if n == self.T and n != self.V else 0
        f = (ctypes.c_double * 4)(*[float(v) for v in field])
        out = ctypes.c_double()
        self.ctx.check(self.lib.dec_rms_error(self.handle, on_tets, _ptr(T, torch.float64, n, "T"), f,
                                              ctypes.byref(out)), "dec_rms_error")
        return out.value

    def dual(self, bc_type, bc_value, side=None, kappa_face=None, cracks=None, limiter=0.0):
        """The system of the paper's own unknowns (temperature per tet, flux per triangle) as a
        DualMesh, assembled and with its boundary data applied; see dec_dual_build.  bc_type per
        vertex: 1 Dirichlet (bc_value the temperature), 2 Neumann (bc_value the outward flux
        density), 0 free; a boundary face takes the kind its three vertices share, else it is
        insulated."""
        return DualMesh(self, bc_type, bc_value, side, kappa_face, cracks, limiter)


class DualMesh(Mesh):
    """A dec_mesh whose rows are the tets of a mesh (dec_dual_build): solve, spmv, csr and fsai
    apply as for vertex meshes; V is the tet count of the source mesh, F its face count."""

    def __init__(self, mesh, bc_type, bc_value, side=None, kappa_face=None, cracks=None, limiter=0.0):
        self.ctx = mesh.ctx
        self.lib = mesh.lib
        n = 0 if cracks is None else int(cracks.shape[0])
        h = ctypes.c_void_p()
        npin = ctypes.c_int64()
        rc = self.lib.dec_dual_build(
            mesh.handle, _ptr(kappa_face, torch.float64, mesh.F, "kappa_face"), n,
            _ptr(cracks, torch.float64, 7 * n, "cracks") if n else None,
            _ptr(bc_type, torch.int8, mesh.V, "bc_type"), _ptr(bc_value, torch.float64, mesh.V, "bc_value"),
            _ptr(side, torch.int8, mesh.V, "side"), float(limiter), ctypes.byref(h), ctypes.byref(npin))
        self.ctx.check(rc, "dec_dual_build")
        self._adopt(h)
        self.n_pinned = npin.value

    def solve(self, T=None, opts=None, check=True, **kw):
        """As Mesh.solve, with the block-Jacobi preconditioner and the A-norm error test unless
        `precond` / `norm` are given: limited faces couple their tets with kappa / limiter, which
        leaves the plain residual of any FP64 vector near eps * kappa / limiter."""
        if opts is None:
            kw.setdefault("precond", DEC_PRECOND_BLOCK)
            kw.setdefault("norm", DEC_NORM_ENERGY)
        return super().solve(T, opts, check, **kw)

    def info(self):
        """dict(faces, limited, blocks, max_block) of dec_dual_info."""
        vals = [ctypes.c_int64() for _ in range(4)]
        self.ctx.check(self.lib.dec_dual_info(self.handle, *[ctypes.byref(v) for v in vals]), "dec_dual_info")
        return dict(zip(("faces", "limited", "blocks", "max_block"), (v.value for v in vals)))

    def faces(self):
        """Device tensors: face_tets [F,2] i32, face_local [F,2] i32, weight [F] f64, cut [F] u8."""
        ft = torch.empty((self.F, 2), dtype=torch.int32, device=self.dev)
        fl = torch.empty((self.F, 2), dtype=torch.int32, device=self.dev)
        w = torch.empty(self.F, dtype=torch.float64, device=self.dev)
        cut = torch.empty(self.F, dtype=torch.uint8, device=self.dev)
        self.ctx.check(self.lib.dec_dual_faces(self.handle, _ptr(ft, torch.int32), _ptr(fl, torch.int32),
                                               _ptr(w, torch.float64), _ptr(cut, torch.uint8)), "dec_dual_faces")
        return ft, fl, w, cut

    def flux(self, T, length=1.0, area=1.0, dT=1.0):
        vals = [ctypes.c_double() for _ in range(4)]
        rc = self.lib.dec_dual_flux(self.handle, _ptr(T, torch.float64, self.V, "T"), length, area, dT,
                                    *[ctypes.byref(v) for v in vals])
        self.ctx.check(rc, "dec_dual_flux")
        k, qi, qo, en = (v.value for v in vals)
        return {"k_eff": k, "q_in": qi, "q_out": qo, "energy": en}


class Server:
    """dec_server: batched solves of many requests, admitted by HBM budget.

    A request is a dict of device tensors: xyz [V,3] f64, tets [T,4] i32,
    kappa [E] f64 (optional), cracks [n,7] f64 (optional), bc_type [V] i8,
    bc_value [V] f64, neumann_f0 [V] f64 (optional), side [V] i8 (optional),
    T_out [V] f64 (optional), T0 [V] f64 (optional warm start), mesh (optional Mesh
    whose topology the server copies instead of building it from xyz and tets),
    and scalars length/area/dT.  The tensors are
    kept referenced until the request's result has been polled.
    """

    def __init__(self, ctx, hbm_budget_bytes, **opts):
        self.ctx = ctx
        self.lib = ctx.lib
        o = _lib.ServerOpts()
        self.lib.dec_server_opts_default(ctypes.byref(o))
        for k, v in opts.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        h = ctypes.c_void_p()
        ctx.check(self.lib.dec_server_create(ctx.handle, int(hbm_budget_bytes), ctypes.byref(o), ctypes.byref(h)),
                  "dec_server_create")
        self.handle = h
        ctx._children.add(self)
        self._keep = {}

    def submit(self, req, user_tag=0):
        mesh = req.get("mesh")
        if mesh is not None:
            V, T = mesh.V, mesh.T
        else:
            V, T = int(req["xyz"].shape[0]), int(req["tets"].shape[0])
        cracks = req.get("cracks")
        n = 0 if cracks is None else int(cracks.shape[0])
        r = _lib.Request()
        r.V, r.T = V, T
        r.xyz = _ptr(req.get("xyz"), torch.float64, 3 * V, "xyz")
        r.tets = _ptr(req.get("tets"), torch.int32, 4 * T, "tets")
        r.mesh = mesh.handle if mesh is not None else None
        r.kappa = _ptr(req.get("kappa"), torch.float64, None, "kappa")
        r.n_cracks = n
        r.cracks = _ptr(cracks, torch.float64, 7 * n, "cracks") if n else None
        r.bc_type = _ptr(req["bc_type"], torch.int8, V, "bc_type")
        r.bc_value = _ptr(req["bc_value"], torch.float64, V, "bc_value")
        r.neumann_f0 = _ptr(req.get("neumann_f0"), torch.float64, V, "neumann_f0")
        r.side = _ptr(req.get("side"), torch.int8, V, "side")
        r.length, r.area, r.dT = (float(req.get(k, 1.0)) for k in ("length", "area", "dT"))
        r.T_out = _ptr(req.get("T_out"), torch.float64, V, "T_out")
        r.T0 = _ptr(req.get("T0"), torch.float64, V, "T0")
        r.user_tag = int(user_tag)
        t = ctypes.c_uint64()
        self.ctx.check(self.lib.dec_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)), "dec_server_submit")
        self._keep[t.value] = req
        return t.value

    def step(self):
        a, p = ctypes.c_int32(), ctypes.c_int32()
        self.ctx.check(self.lib.dec_server_step(self.handle, ctypes.byref(a), ctypes.byref(p)), "dec_server_step")
        return a.value, p.value

    def poll(self, max_results=256):
        buf = (_lib.Result * max_results)()
        n = ctypes.c_int32()
        self.ctx.check(self.lib.dec_server_poll(self.handle, buf, max_results, ctypes.byref(n)), "dec_server_poll")
        out = []
        for i in range(n.value):
            d = buf[i].as_dict()
            d["request"] = self._keep.pop(d["ticket"], None)
            out.append(d)
        return out

    def cancel(self, ticket):
        return self.lib.dec_server_cancel(self.handle, int(ticket))

    def stats(self):
        """Batched inner iterations so far: replay time (ms), algorithmic bytes, system-iterations, and the
        batched product's variant per precision (entry pairs in flight, non-temporal loads, columns first)."""
        c = _lib.ServerCounters()
        self.ctx.check(self.lib.dec_server_stats(self.handle, ctypes.byref(c)), "dec_server_stats")
        v, h, o = list(c.variant), list(c.host_ms), list(c.order)
        return {"batch_ms": c.batch_ms, "batch_bytes": c.batch_bytes, "batch_iterations": c.batch_iterations,
                "variant_fp64": {"unroll": v[0], "nontemporal": v[1], "columns_first": o[0]},
                "variant_fp32": {"unroll": v[2], "nontemporal": v[3], "columns_first": o[1]},
                "host_ms": {"launch": h[0], "admit": h[1], "wait": h[2], "refine": h[3]}, "steps": c.steps}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dec_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
