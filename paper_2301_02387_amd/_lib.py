"""ctypes binding of libmh.so; names follow include/mh.h."""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
MH_OK, MH_NOT_CONVERGED = 0, 1
_NAMES = {-1: "INVALID_ARG", -2: "OOM", -3: "HIP_ERROR", -4: "SINGULAR_RDM", -5: "NONFINITE",
          -6: "UNSUPPORTED"}

EXPORTS = ["mh_mesh_create", "mh_mesh_info_get", "mh_mesh_node_coords", "mh_mesh_constraints",
           "mh_mesh_destroy", "mh_op_create", "mh_op_destroy", "mh_fill_hanging", "mh_mass_solve", "mh_mass_solve_noalloc",
           "mh_h1_apply", "mh_poisson_pairs", "mh_ci_rdms", "mh_freeze", "mh_rhs_apply",
           "mh_arnoldi_step", "mh_propagate", "mh_op_sizes_get", "mh_kernel_timing", "mh_tune",
           "mh_propagate_adjoint", "mh_batch_create", "mh_batch_layout", "mh_set_allocator", "mh_last_error"]


class MHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mh error {code} ({_NAMES.get(code, '?')}): {msg}")
        self.code = code


class _Ball(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("radius", C.c_double), ("levels", C.c_int32)]


class _MeshDesc(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("n_coarse", C.c_int32), ("p", C.c_int32),
                ("n_balls", C.c_int32), ("balls", C.POINTER(_Ball)),
                ("n_kelly", C.c_int32), ("kelly_nuclei", C.POINTER(C.c_double)), ("kelly_tol", C.c_double),
                ("kelly_soft", C.c_double), ("kelly_max_level", C.c_int32)]


class _MeshInfo(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_full", C.c_int64), ("n_dof", C.c_int64), ("n_hang", C.c_int64),
                ("n_bnd", C.c_int64), ("n_masters", C.c_int64), ("hang_nnz", C.c_int64), ("p", C.c_int32),
                ("max_level", C.c_int32), ("level_counts", C.c_int64 * 16), ("kelly_rounds", C.c_int32)]


class _OpDesc(C.Structure):
    _fields_ = [("n_nuclei", C.c_int32), ("charges", C.POINTER(C.c_double)),
                ("positions", C.POINTER(C.c_double)), ("n_orb", C.c_int32), ("n_alpha", C.c_int32),
                ("n_beta", C.c_int32), ("polarization", C.c_double * 3), ("lmax_bc", C.c_int32),
                ("poisson_rtol", C.c_double), ("poisson_maxit", C.c_int32), ("rdm_eps", C.c_double),
                ("gauge", C.c_int32), ("krylov_tol", C.c_double), ("ecs_theta", C.c_double),
                ("ecs_inner", C.c_double * 3)]


class _Obs(C.Structure):
    _fields_ = [("dipole", C.POINTER(C.c_double)), ("energy", C.POINTER(C.c_double)),
                ("err_est", C.POINTER(C.c_double)), ("ortho", C.POINTER(C.c_double)),
                ("cg_iters", C.POINTER(C.c_int32)), ("momentum", C.POINTER(C.c_double)),
                ("krylov_dim", C.POINTER(C.c_int32))]


class _Sizes(C.Structure):
    _fields_ = [("n_dof", C.c_int64), ("n_ext", C.c_int64), ("n_full", C.c_int64), ("n_ci", C.c_int64),
                ("n_orb", C.c_int32), ("n_pair_cols", C.c_int32), ("n_poisson_nnz", C.c_int64),
                ("n_inst", C.c_int32)]


_lib = None


def lib_path():
    return os.path.join(_HERE, "libmh.so")


def load_library():
    """Load libmh.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2301_02387_amd.build`")
    # PyTorch carries its own HIP runtime (soname libamdhip64.so.7).  Loading
    # torch first makes libmh.so bind to that same runtime, so that torch's
    # device pointers and streams are valid in the library; loading libmh.so
    # first would bring a second runtime into the process.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.mh_last_error.restype = C.c_char_p
    lib.mh_mesh_create.argtypes = [C.POINTER(_MeshDesc), C.POINTER(vp)]
    lib.mh_mesh_info_get.argtypes = [vp, C.POINTER(_MeshInfo)]
    lib.mh_mesh_node_coords.argtypes = [vp, vp]
    lib.mh_mesh_constraints.argtypes = [vp, vp, vp, vp]
    lib.mh_mesh_cells.argtypes = [vp, vp, vp, vp]
    lib.mh_mesh_destroy.argtypes = [vp]
    lib.mh_op_create.argtypes = [vp, C.POINTER(_OpDesc), vp, C.POINTER(vp)]
    lib.mh_op_destroy.argtypes = [vp]
    lib.mh_op_sizes_get.argtypes = [vp, C.POINTER(_Sizes)]
    lib.mh_fill_hanging.argtypes = [vp, vp, vp]
    lib.mh_mass_solve.argtypes = [vp, vp, vp, vp]
    lib.mh_mass_solve_noalloc.argtypes = [vp, vp, vp, vp]
    lib.mh_h1_apply.argtypes = [vp, vp, C.c_double, vp, vp]
    lib.mh_poisson_pairs.argtypes = [vp, vp, vp, C.c_int32, C.POINTER(C.c_int32), vp]
    lib.mh_ci_rdms.argtypes = [vp, vp, vp, vp, vp]
    lib.mh_freeze.argtypes = [vp, vp, vp, vp, C.c_double, vp, vp]
    lib.mh_rhs_apply.argtypes = [vp, vp, vp, vp]
    lib.mh_arnoldi_step.argtypes = [vp, vp, C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_int32), vp]
    lib.mh_propagate.argtypes = [vp, vp, vp, vp, vp, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                 C.POINTER(_Obs), vp]
    lib.mh_kernel_timing.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.mh_tune.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    lib.mh_propagate_adjoint.argtypes = [vp, vp, vp, vp, vp, C.c_int32, C.c_double, C.c_int32, vp, vp,
                                         C.c_int32, C.c_int32, vp]
    lib.mh_batch_create.argtypes = [vp, vp, vp, C.c_int32, vp, C.POINTER(vp)]
    lib.mh_batch_layout.argtypes = [vp, vp]
    lib.mh_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
    for name in EXPORTS:
        if name != "mh_last_error":
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)
_ALLOCATORS = []    # every registered pair of callbacks, kept alive for the handles that use them


def set_allocator(alloc=None, free=None):
    """Register the device allocator of the library's own workspaces
    (mh_set_allocator): alloc(nbytes) -> int device address (0 on failure),
    free(address, nbytes).  alloc="torch" takes torch's caching allocator on
    the current device and stream.  No arguments restore hipMalloc/hipFree.
    Handles return their buffers to the functions that made them, so every
    pair registered stays referenced for the life of the process."""
    lib = load_library()
    if alloc is None and free is None:
        _check(lib.mh_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
        return
    if alloc == "torch":
        import torch

        def alloc(nbytes):
            return torch.cuda.caching_allocator_alloc(int(nbytes))

        def free(ptr, nbytes):
            torch.cuda.caching_allocator_delete(int(ptr))

    def _a(nbytes, ctx):
        try:
            return int(alloc(nbytes)) or None
        except Exception:   # reported to the library as a failed allocation
            return None

    def _f(ptr, nbytes, ctx):
        try:
            free(ptr, nbytes)
        except Exception:   # nothing to report from a release
            pass

    cbs = (_ALLOC_FN(_a), _FREE_FN(_f))
    _ALLOCATORS.append(cbs)
    _check(lib.mh_set_allocator(cbs[0], cbs[1], None))


def _check(rc, allow_nc=False):
    if rc == MH_OK or (allow_nc and rc == MH_NOT_CONVERGED):
        return rc
    raise MHError(rc, _lib.mh_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


class Mesh:
    """Octree mesh (host); see mh_mesh_create."""

    def __init__(self, lo, hi, n_coarse, p, balls, kelly=None):
        """kelly: optional dict(nuclei=[(Z, (x, y, z))], tol, soft, max_level)."""
        lib = load_library()
        arr = (_Ball * max(1, len(balls)))()
        for i, b in enumerate(balls):
            arr[i].center[:] = list(map(float, b["center"]))
            arr[i].radius = float(b["radius"])
            arr[i].levels = int(b["levels"])
        kn = np.zeros((1, 4))
        nk, ktol, ksoft, klev = 0, 0.0, 0.0, 0
        if kelly:
            kn = np.ascontiguousarray([[float(z), *map(float, r)] for z, r in kelly["nuclei"]], dtype=np.float64)
            nk, ktol, ksoft, klev = len(kn), float(kelly["tol"]), float(kelly["soft"]), int(kelly["max_level"])
        self._kn = kn
        desc = _MeshDesc(float(lo), float(hi), int(n_coarse), int(p), len(balls), arr, nk,
                         kn.ctypes.data_as(C.POINTER(C.c_double)), ktol, ksoft, klev)
        h = C.c_void_p()
        _check(lib.mh_mesh_create(C.byref(desc), C.byref(h)))
        self._h = h
        info = _MeshInfo()
        _check(lib.mh_mesh_info_get(h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in _MeshInfo._fields_ if k != "level_counts"}
        self.info["level_counts"] = list(info.level_counts[:info.max_level + 1])

    @classmethod
    def from_workload(cls, w):
        return cls(w["lo"], w["hi"], w["n_coarse"], w["p"], w["balls"], w.get("kelly"))

    def coords(self):
        out = np.zeros((self.info["n_full"], 3))
        _check(_lib.mh_mesh_node_coords(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def cells(self):
        """(nodes [n_cells][(p+1)^3] int32, level [n_cells] int32, origin [n_cells][3]) in library order."""
        nc, P3 = self.info["n_cells"], (self.info["p"] + 1) ** 3
        nodes = np.zeros((nc, P3), dtype=np.int32)
        level = np.zeros(nc, dtype=np.int32)
        origin = np.zeros((nc, 3))
        _check(_lib.mh_mesh_cells(self._h, nodes.ctypes.data_as(C.c_void_p), level.ctypes.data_as(C.c_void_p),
                                  origin.ctypes.data_as(C.c_void_p)))
        return nodes, level, origin

    def constraints(self):
        nh, nnz = self.info["n_hang"], self.info["hang_nnz"]
        ptr = np.zeros(nh + 1, dtype=np.int64)
        col = np.zeros(max(1, nnz), dtype=np.int64)
        w = np.zeros(max(1, nnz))
        _check(_lib.mh_mesh_constraints(self._h, ptr.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p),
                                        w.ctypes.data_as(C.c_void_p)))
        return ptr, col[:nnz], w[:nnz]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mh_mesh_destroy(self._h)
            self._h = None


GAUGES = {"length": 0, "velocity": 1}


def _op_desc(nuclei, n_orb, n_alpha, n_beta, polarization, lmax_bc, poisson_rtol, poisson_maxit, rdm_eps,
             gauge="length", krylov_tol=0.0, ecs=None):
    """ecs: None or (theta, (Rx, Ry, Rz)), exterior complex scaling."""
    Z = np.array([z for z, _ in nuclei], dtype=np.float64)
    R = np.ascontiguousarray(np.array([r for _, r in nuclei], dtype=np.float64).reshape(-1, 3))
    theta, inner = (0.0, (0.0, 0.0, 0.0)) if ecs is None else (float(ecs[0]), tuple(map(float, ecs[1])))
    desc = _OpDesc(len(nuclei), Z.ctypes.data_as(C.POINTER(C.c_double)), R.ctypes.data_as(C.POINTER(C.c_double)),
                   int(n_orb), int(n_alpha), int(n_beta), (C.c_double * 3)(*polarization), int(lmax_bc),
                   float(poisson_rtol), int(poisson_maxit), float(rdm_eps), GAUGES[gauge], float(krylov_tol),
                   theta, (C.c_double * 3)(*inner))
    return desc, (Z, R)


class Operator:
    """Operator set-up and device entry points (see include/mh.h)."""

    def __init__(self, mesh, nuclei, n_orb, n_alpha, n_beta, polarization=(0.0, 0.0, 1.0), lmax_bc=12,
                 poisson_rtol=1e-12, poisson_maxit=5000, rdm_eps=1e-10, gauge="length", krylov_tol=0.0,
                 stream=None, ecs=None):
        lib = load_library()
        desc, keep = _op_desc(nuclei, n_orb, n_alpha, n_beta, polarization, lmax_bc, poisson_rtol,
                              poisson_maxit, rdm_eps, gauge, krylov_tol, ecs)
        h = C.c_void_p()
        _check(lib.mh_op_create(mesh._h, C.byref(desc), _stream(stream), C.byref(h)))
        self._attach(h, [mesh])

    @classmethod
    def batch(cls, meshes, nuclei_list, n_orb, n_alpha, n_beta, field_scale=None, polarization=(0.0, 0.0, 1.0),
              lmax_bc=12, poisson_rtol=1e-12, poisson_maxit=5000, rdm_eps=1e-10, gauge="length", krylov_tol=0.0,
              stream=None, ecs=None):
        """Batch of independent instances (mh_batch_create): one mesh and one
        molecule per instance, one shared orbital/electron space.  ecs: None,
        one (theta, inner) for every instance, or a list of them (or None)
        per instance."""
        lib = load_library()
        ni = len(meshes)
        if len(nuclei_list) != ni:
            raise ValueError("one nuclei list per mesh")
        descs = (_OpDesc * ni)()
        keep = []
        for i, nuc in enumerate(nuclei_list):
            ei = ecs[i] if isinstance(ecs, list) else ecs
            d, k = _op_desc(nuc, n_orb, n_alpha, n_beta, polarization, lmax_bc, poisson_rtol, poisson_maxit,
                            rdm_eps, gauge, krylov_tol, ei)
            descs[i] = d
            keep.append(k)
        hs = (C.c_void_p * ni)(*[m._h.value for m in meshes])
        fs = np.ascontiguousarray(np.ones(ni) if field_scale is None else field_scale, dtype=np.float64)
        if fs.shape != (ni,):
            raise ValueError("field_scale must have one entry per instance")
        h = C.c_void_p()
        _check(lib.mh_batch_create(C.cast(hs, C.c_void_p), C.cast(descs, C.c_void_p),
                                   fs.ctypes.data_as(C.c_void_p), ni, _stream(stream), C.byref(h)))
        self = cls.__new__(cls)
        self._attach(h, list(meshes))
        return self

    def _attach(self, h, meshes):
        self._h = h
        self.meshes = meshes
        self.mesh = meshes[0]
        sz = _Sizes()
        _check(_lib.mh_op_sizes_get(h, C.byref(sz)))
        self.n_dof, self.n_ext, self.n_full, self.n_ci = sz.n_dof, sz.n_ext, sz.n_full, sz.n_ci
        self.n_orb, self.n_pair_cols = sz.n_orb, sz.n_pair_cols
        self.n_poisson_nnz = sz.n_poisson_nnz
        self.n_inst = sz.n_inst

    def layout(self):
        """Per instance: N, N_E, N_F, oE, oF, Poisson nnz (mh_batch_layout)."""
        out = np.zeros((self.n_inst, 6), dtype=np.int64)
        _check(_lib.mh_batch_layout(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mh_op_destroy(self._h)
            self._h = None

    def _need(self, t, rows, cols, dtype):
        import torch
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
            raise ValueError("expected a contiguous CUDA tensor of dtype %s" % dtype)
        if t.numel() != rows * cols:
            raise ValueError(f"expected {rows}x{cols} elements, got {tuple(t.shape)}")

    def fill_hanging(self, x, stream=None):
        import torch
        self._need(x, self.n_ext, self.n_orb, torch.complex128)
        _check(_lib.mh_fill_hanging(self._h, _ptr(x), _stream(stream)))

    def mass_solve(self, f, c, stream=None):
        import torch
        self._need(c, self.n_ext, self.n_orb, torch.complex128)
        if f.numel() < self.n_dof * self.n_orb:
            raise ValueError("f too small")
        _check(_lib.mh_mass_solve(self._h, _ptr(f), _ptr(c), _stream(stream)))

    def mass_solve_noalloc(self, f, c, stream=None):
        """mh_mass_solve through the library's static device scratch (no allocation)."""
        import torch
        self._need(c, self.n_ext, self.n_orb, torch.complex128)
        if f.numel() < self.n_dof * self.n_orb:
            raise ValueError("f too small")
        _check(_lib.mh_mass_solve_noalloc(self._h, _ptr(f), _ptr(c), _stream(stream)))

    def h1_apply(self, c, E, f, stream=None):
        import torch
        self._need(c, self.n_ext, self.n_orb, torch.complex128)
        self._need(f, self.n_dof if self.n_inst == 1 else self.n_ext, self.n_orb, torch.complex128)
        _check(_lib.mh_h1_apply(self._h, _ptr(c), float(E), _ptr(f), _stream(stream)))

    def poisson_pairs(self, phi, W, warm=False, stream=None):
        import torch
        self._need(phi, self.n_ext, self.n_orb, torch.complex128)
        self._need(W, self.n_full, self.n_pair_cols, torch.float64)
        it = C.c_int32(0)
        rc = _check(_lib.mh_poisson_pairs(self._h, _ptr(phi), _ptr(W), int(bool(warm)), C.byref(it),
                                          _stream(stream)), allow_nc=True)
        return it.value, rc

    def ci_rdms(self, Ci, gamma, Gamma, stream=None):
        _check(_lib.mh_ci_rdms(self._h, _ptr(Ci), _ptr(gamma), _ptr(Gamma), _stream(stream)))

    def freeze(self, phi, gamma, Gamma, E, W, stream=None):
        _check(_lib.mh_freeze(self._h, _ptr(phi), _ptr(gamma), _ptr(Gamma), float(E), _ptr(W), _stream(stream)))

    def rhs_apply(self, v, Gv, stream=None):
        import torch
        self._need(v, self.n_ext, self.n_orb, torch.complex128)
        self._need(Gv, self.n_ext, self.n_orb, torch.complex128)
        _check(_lib.mh_rhs_apply(self._h, _ptr(v), _ptr(Gv), _stream(stream)))

    def arnoldi_step(self, phi, tau, m, stream=None):
        import torch
        self._need(phi, self.n_ext, self.n_orb, torch.complex128)
        tau = complex(tau)
        err = C.c_double(0)
        mu = C.c_int32(0)
        _check(_lib.mh_arnoldi_step(self._h, _ptr(phi), tau.real, tau.imag, int(m), C.byref(err), C.byref(mu),
                                    _stream(stream)))
        return err.value, mu.value

    def propagate(self, phi, Ci, W, E_steps, dt, m=12, imaginary=False, final=True, graph=False, graph_step=False,
                  stream=None):
        """Records are [n_steps + 1] for one instance, [n_steps + 1][n_inst] for a batch.
        graph: replay the part of each step after the Poisson solve from a HIP
        graph; graph_step: replay whole steps (MH_PROP_GRAPH_STEP)."""
        import torch
        self._need(phi, self.n_ext, self.n_orb, torch.complex128)
        self._need(W, self.n_full, self.n_pair_cols, torch.float64)
        self._need(Ci, self.n_inst, self.n_ci, torch.complex128)
        E = np.ascontiguousarray(E_steps, dtype=np.float64)
        n_steps = len(E) - 1
        shape = (n_steps + 1,) if self.n_inst == 1 else (n_steps + 1, self.n_inst)
        rec = {k: np.zeros(shape) for k in ("dipole", "energy", "err_est", "ortho", "momentum")}
        rec["cg_iters"] = np.zeros(n_steps + 1, dtype=np.int32)
        rec["krylov_dim"] = np.zeros(shape, dtype=np.int32)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))  # noqa: E731
        obs = _Obs(dp(rec["dipole"]), dp(rec["energy"]), dp(rec["err_est"]), dp(rec["ortho"]),
                   ip(rec["cg_iters"]), dp(rec["momentum"]), ip(rec["krylov_dim"]))
        rc = _check(_lib.mh_propagate(self._h, _ptr(phi), _ptr(Ci), _ptr(W), E.ctypes.data_as(C.c_void_p),
                                      n_steps, float(dt), int(m),
                                      (1 if imaginary else 0) | (0 if final else 2) | (4 if graph else 0)
                                      | (8 if graph_step else 0),
                                      C.byref(obs),
                                      _stream(stream)), allow_nc=True)
        rec["status"] = rc
        return rec

    def kernel_timing(self, which, enable):
        avg = C.c_double(0)
        cnt = C.c_int64(0)
        _check(_lib.mh_kernel_timing(self._h, int(which), int(bool(enable)), C.byref(avg), C.byref(cnt)))
        return avg.value, cnt.value

    def tune(self, which, sched, grid_cap):
        """Select the launch schedule of operator kernel `which` (mh_tune)."""
        _check(_lib.mh_tune(self._h, int(which), int(sched), int(grid_cap)))

    def propagate_adjoint(self, phi0, Ci0, W, E_steps, dt, dJ_dd, m=12, n_quad=6, ckpt_stride=0, stream=None):
        """dJ/dE_k for the dipole record of propagate (mh_propagate_adjoint)."""
        import torch
        self._need(phi0, self.n_ext, self.n_orb, torch.complex128)
        E = np.ascontiguousarray(E_steps, dtype=np.float64)
        g = np.ascontiguousarray(dJ_dd, dtype=np.float64)
        n_steps = len(E) - 1
        if len(g) != n_steps + 1:
            raise ValueError("dJ_dd must have one entry per dipole record")
        out = np.zeros(n_steps)
        rc = _check(_lib.mh_propagate_adjoint(self._h, _ptr(phi0), _ptr(Ci0), _ptr(W), E.ctypes.data_as(C.c_void_p),
                                              n_steps, float(dt), int(m), g.ctypes.data_as(C.c_void_p),
                                              out.ctypes.data_as(C.c_void_p), int(n_quad), int(ckpt_stride),
                                              _stream(stream)), allow_nc=True)
        if rc == MH_NOT_CONVERGED:
            import warnings
            warnings.warn("a Poisson solve of the adjoint stopped at the iteration cap")
        return out
