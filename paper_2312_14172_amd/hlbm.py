"""Thin ctypes binding of ``libhlbm.so`` (the C ABI in ``include/hlbm.h``).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch supplies the device workspace and the stream.  Importing this module
does not load the library; the first use does, and it raises if the built
library is missing (build it with ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhlbm.so")

HLBM_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "EUNSTABLE", -6: "EUNSUPPORTED"}
BC_PERIODIC, BC_WALL = 0, 1
FP64, FP32, FP16S = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16s": FP16S}
FIELD_RHO, FIELD_U, FIELD_U_PHYS, FIELD_SOLID = 1, 2, 4, 8

EXPORTED = ["hlbm_workspace_size", "hlbm_init", "hlbm_destroy", "hlbm_set_particles",
            "hlbm_set_fields", "hlbm_step", "hlbm_set_fluid_accel", "hlbm_set_contact", "hlbm_set_mesh",
            "hlbm_get_forces",
            "hlbm_get_fields", "hlbm_get_mean_velocity",
            "hlbm_num_particles", "hlbm_profile_begin", "hlbm_profile_end", "hlbm_mlp_set_params",
            "hlbm_mlp_get_params", "hlbm_mlp_eval", "hlbm_mlp_gradient", "hlbm_train_indicator",
            "hlbm_set_indicator", "hlbm_mlp_train_step", "hlbm_mlp_samples", "hlbm_mlp_gradient_noalloc",
            "hlbm_last_error"]
MLP_NPARAM = 8641
INDICATOR_EXACT, INDICATOR_LEARNED = 0, 1


class hlbm_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 3), ("precision", ctypes.c_int32),
                ("max_particles", ctypes.c_int32), ("tau", ctypes.c_double),
                ("eps", ctypes.c_double), ("rho_f", ctypes.c_double),
                ("gravity", ctypes.c_double * 3), ("fluid_accel", ctypes.c_double * 3),
                ("stream", ctypes.c_void_p), ("learned", ctypes.c_int32),
                ("learned_samples", ctypes.c_int32), ("learned_max_circumradius", ctypes.c_double),
                ("max_mesh_triangles", ctypes.c_int32), ("coupling", ctypes.c_int32)]


class hlbm_train_opts(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32), ("holdout", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("lr_final", ctypes.c_double), ("box", ctypes.c_double), ("band", ctypes.c_double),
                ("clip", ctypes.c_double), ("band_share", ctypes.c_double),
                ("gate_rms", ctypes.c_double), ("gate_max", ctypes.c_double),
                ("ref_circumradius", ctypes.c_double), ("seed", ctypes.c_uint64)]


class hlbm_train_report(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("rms_err", ctypes.c_double), ("max_err", ctypes.c_double),
                ("train_ms", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("accepted", ctypes.c_int32)]


# byte layout of struct hlbm_particle
HLBM_PARTICLE = np.dtype([("pos", "<f8", 3), ("quat", "<f8", 4), ("vel", "<f8", 3),
                          ("omega", "<f8", 3), ("mass", "<f8"), ("volume", "<f8"),
                          ("inertia", "<f8", 3), ("param", "<f8", 3), ("shape", "<i4"),
                          ("flags", "<i4")])


class HLBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libhlbm.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        cfgp = ctypes.POINTER(hlbm_config)
        L.hlbm_workspace_size.argtypes = [cfgp, ctypes.POINTER(ctypes.c_size_t)]
        L.hlbm_init.argtypes = [cfgp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.hlbm_destroy.argtypes = [vp]
        L.hlbm_set_particles.argtypes = [vp, i32, vp]
        L.hlbm_set_fields.argtypes = [vp, vp, vp]
        L.hlbm_step.argtypes = [vp, i32]
        L.hlbm_set_fluid_accel.argtypes = [vp, vp]
        L.hlbm_set_contact.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.hlbm_set_mesh.argtypes = [vp, vp, i32, vp, i32]
        L.hlbm_get_forces.argtypes = [vp, vp, vp, vp]
        L.hlbm_get_fields.argtypes = [vp, ctypes.c_uint32, i32, vp, i32]
        L.hlbm_get_mean_velocity.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_int64)]
        L.hlbm_num_particles.argtypes = [vp, ctypes.POINTER(i32)]
        L.hlbm_profile_begin.argtypes = [vp]
        L.hlbm_profile_end.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
        L.hlbm_mlp_set_params.argtypes = [vp, i32, vp]
        L.hlbm_mlp_get_params.argtypes = [vp, i32, vp]
        L.hlbm_mlp_eval.argtypes = [vp, i32, i32, vp, vp]
        L.hlbm_mlp_gradient.argtypes = [vp, i32, i32, vp, vp, vp, vp]
        L.hlbm_train_indicator.argtypes = [vp, i32, vp, ctypes.POINTER(hlbm_train_opts),
                                           ctypes.POINTER(hlbm_train_report)]
        L.hlbm_set_indicator.argtypes = [vp, i32, i32]
        L.hlbm_mlp_gradient_noalloc.argtypes = [vp, i32, vp, vp, vp]
        L.hlbm_mlp_train_step.argtypes = [vp, i32, i32, vp, vp, ctypes.c_double, i32, vp, vp]
        L.hlbm_mlp_samples.argtypes = [vp, i32, vp, ctypes.c_uint64, i32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, vp]
        L.hlbm_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name != "hlbm_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != HLBM_OK:
        raise HLBMError(rc, lib().hlbm_last_error().decode())


COUPLINGS = {"hlbm": 0, "psm": 1}


def make_config(n, bc=(0, 0, 0), tau=0.8, precision="fp64", max_particles=0, eps=0.5, rho_f=1.0,
                gravity=(0.0, 0.0, 0.0), fluid_accel=(0.0, 0.0, 0.0), stream=None,
                learned_max_circumradius=0.0, learned_samples=0, max_mesh_triangles=0, coupling="hlbm"):
    c = hlbm_config()
    c.nx, c.ny, c.nz = (int(v) for v in n)
    c.bc = (ctypes.c_int32 * 3)(*[int(b) for b in bc])
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.max_particles = int(max_particles)
    c.tau, c.eps, c.rho_f = float(tau), float(eps), float(rho_f)
    c.gravity = (ctypes.c_double * 3)(*gravity)
    c.fluid_accel = (ctypes.c_double * 3)(*fluid_accel)
    c.stream = stream
    c.learned = 1 if learned_max_circumradius > 0 else 0
    c.learned_samples = int(learned_samples)
    c.learned_max_circumradius = float(learned_max_circumradius)
    c.max_mesh_triangles = int(max_mesh_triangles)
    c.coupling = COUPLINGS[coupling] if isinstance(coupling, str) else int(coupling)
    return c


def to_particle_records(particles) -> np.ndarray:
    """Copy a record array with the fields of ``struct hlbm_particle`` (by
    name) into the ABI's byte layout."""
    out = np.zeros(len(particles), dtype=HLBM_PARTICLE)
    for name in HLBM_PARTICLE.names:
        out[name] = particles[name]
    return out


def mlp_gradient_noalloc(theta, samples, grad, stream=None):
    """hlbm_mlp_gradient_noalloc on device tensors: theta [8641] float32,
    samples [n, 4] float32 (x, y, z, target), grad [8642] float32 (gradient,
    then the sum of squared errors); queued on the stream (torch's current
    one by default), not synchronised."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(theta.device)
    for t in (theta, samples, grad):
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    assert theta.numel() == MLP_NPARAM and grad.numel() == MLP_NPARAM + 1 and samples.shape[-1] == 4
    _check(lib().hlbm_mlp_gradient_noalloc(ctypes.c_void_p(theta.data_ptr()), int(samples.shape[0]),
                                           ctypes.c_void_p(samples.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                           ctypes.c_void_p(s.cuda_stream)))


class Simulation:
    """One HLBM context on the current HIP device."""

    def __init__(self, n, bc=(0, 0, 0), tau=0.8, precision="fp64", max_particles=0, eps=0.5,
                 rho_f=1.0, gravity=(0.0, 0.0, 0.0), fluid_accel=(0.0, 0.0, 0.0), device=None,
                 stream=None, learned_max_circumradius=0.0, learned_samples=0, max_mesh_triangles=0,
                 coupling="hlbm"):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n = tuple(int(v) for v in n)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.cfg = make_config(n, bc, tau, precision, max_particles, eps, rho_f, gravity,
                               fluid_accel, ctypes.c_void_p(self.stream.cuda_stream),
                               learned_max_circumradius, learned_samples, max_mesh_triangles, coupling)
        nbytes = ctypes.c_size_t(0)
        _check(lib().hlbm_workspace_size(ctypes.byref(self.cfg), ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self._ctx = ctypes.c_void_p()
        _check(lib().hlbm_init(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                               nbytes.value, ctypes.byref(self._ctx)))
        self.num_particles = 0

    def close(self):
        if self._ctx:
            _check(lib().hlbm_destroy(self._ctx))
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_particles(self, particles):
        recs = to_particle_records(particles)
        _check(lib().hlbm_set_particles(self._ctx, len(recs),
                                        recs.ctypes.data if len(recs) else None))
        self.num_particles = len(recs)

    def set_fields(self, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(3, -1)
        _check(lib().hlbm_set_fields(self._ctx, None if r is None else r.ctypes.data,
                                     None if v is None else v.ctypes.data))

    def step(self, nsteps=1):
        _check(lib().hlbm_step(self._ctx, int(nsteps)))

    def profile_begin(self):
        _check(lib().hlbm_profile_begin(self._ctx))

    def profile_end(self):
        """Summed HIP-event time (ms) and count of the collide launches."""
        ms = ctypes.c_double(0)
        cnt = ctypes.c_int64(0)
        _check(lib().hlbm_profile_end(self._ctx, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def set_mesh(self, vertices, triangles):
        """Closed triangle mesh of HLBM_MESH particles (unit scale, body frame,
        counter-clockwise seen from outside)."""
        v = np.ascontiguousarray(vertices, dtype=np.float32).reshape(-1, 3)
        t = np.ascontiguousarray(triangles, dtype=np.int32).reshape(-1, 3)
        _check(lib().hlbm_set_mesh(self._ctx, v.ctypes.data, len(v), t.ctypes.data, len(t)))

    def set_fluid_accel(self, accel):
        """Fluid body acceleration (outside the solid) from the next step on."""
        a = np.ascontiguousarray(accel, dtype=np.float64).reshape(3)
        _check(lib().hlbm_set_fluid_accel(self._ctx, a.ctypes.data))

    def set_contact(self, range_, stiffness, wall_stiffness=0.0):
        """Contact repulsion (range, pair stiffness, wall stiffness) from the
        next step on, for spheres and non-spherical shapes; range 0 turns it
        off."""
        _check(lib().hlbm_set_contact(self._ctx, float(range_), float(stiffness), float(wall_stiffness)))

    def get_forces(self):
        n = self.num_particles
        F = np.zeros((max(n, 1), 3))
        T = np.zeros((max(n, 1), 3))
        st = np.zeros(max(n, 1), dtype=HLBM_PARTICLE)
        _check(lib().hlbm_get_forces(self._ctx, F.ctypes.data, T.ctypes.data, st.ctypes.data))
        return F[:n], T[:n], st[:n]

    def get_fields(self, mask=FIELD_RHO | FIELD_U | FIELD_U_PHYS | FIELD_SOLID, on_device=False,
                   dtype="fp64"):
        """Fields as FP64 (dtype "fp64") or FP32 ("fp32") planes: a device
        tensor [planes, ncells] with on_device, else a dict of numpy arrays."""
        planes = (1 if mask & 1 else 0) + (3 if mask & 2 else 0) + (3 if mask & 4 else 0) + \
                 (1 if mask & 8 else 0)
        code = {"fp64": FP64, "fp32": FP32}[dtype]
        if on_device:
            tdt = self.torch.float64 if dtype == "fp64" else self.torch.float32
            out = self.torch.empty((planes, self.N), dtype=tdt, device=self.device)
            _check(lib().hlbm_get_fields(self._ctx, mask, code, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        out = np.zeros((planes, self.N), dtype=np.float64 if dtype == "fp64" else np.float32)
        _check(lib().hlbm_get_fields(self._ctx, mask, code, out.ctypes.data, 0))
        res = {}
        k = 0
        if mask & 1:
            res["rho"] = out[k]; k += 1
        if mask & 2:
            res["u"] = out[k:k + 3]; k += 3
        if mask & 4:
            res["u_phys"] = out[k:k + 3]; k += 3
        if mask & 8:
            res["B"] = out[k]
        return res

    def get_mean_velocity(self):
        """(mean u_phys over all cells [3], mean u_phys over pure-fluid cells
        [3], number of pure-fluid cells), reduced in FP64 on the device."""
        a = np.zeros(3)
        b = np.zeros(3)
        n = ctypes.c_int64(0)
        _check(lib().hlbm_get_mean_velocity(self._ctx, a.ctypes.data, b.ctypes.data, ctypes.byref(n)))
        return a, b, n.value

    # ---- learned indicator ---------------------------------------------
    def mlp_set_params(self, shape, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.size == MLP_NPARAM
        _check(lib().hlbm_mlp_set_params(self._ctx, int(shape), th.ctypes.data))

    def mlp_get_params(self, shape):
        th = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(lib().hlbm_mlp_get_params(self._ctx, int(shape), th.ctypes.data))
        return th

    def mlp_eval(self, shape, pts):
        p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        out = np.zeros(len(p))
        _check(lib().hlbm_mlp_eval(self._ctx, int(shape), len(p), p.ctypes.data, out.ctypes.data))
        return out

    def mlp_gradient(self, shape, pts, target):
        p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        t = np.ascontiguousarray(target, dtype=np.float64).reshape(-1)
        g = np.zeros(MLP_NPARAM)
        loss = ctypes.c_double(0)
        _check(lib().hlbm_mlp_gradient(self._ctx, int(shape), len(p), p.ctypes.data, t.ctypes.data,
                                       g.ctypes.data, ctypes.byref(loss)))
        return g, loss.value

    def mlp_train_step(self, shape, pts, target, lr, step):
        """Gradient on (pts, target), then one Adam step (the step-th);
        returns (gradient, loss)."""
        p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        t = np.ascontiguousarray(target, dtype=np.float64).reshape(-1)
        g = np.zeros(MLP_NPARAM)
        loss = ctypes.c_double(0)
        _check(lib().hlbm_mlp_train_step(self._ctx, int(shape), len(p), p.ctypes.data, t.ctypes.data,
                                         float(lr), int(step), g.ctypes.data, ctypes.byref(loss)))
        return g, loss.value

    def mlp_samples(self, shape, param, n, seed=4, box=1.1, band=0.1, clip=0.25, band_share=0.8):
        """The training samples [n, 4] (x, y, z, clipped signed distance) the
        GPU generator draws, in normalised units."""
        prm = np.ascontiguousarray(list(param) + [0.0] * (3 - len(param)), dtype=np.float64)
        out = np.zeros((int(n), 4))
        _check(lib().hlbm_mlp_samples(self._ctx, int(shape), prm.ctypes.data, int(seed), int(n), float(box),
                                      float(band), float(clip), float(band_share), out.ctypes.data))
        return out

    def train_indicator(self, shape, param, samples=1_000_000, holdout=100_000, iterations=3000,
                        batch=8192, lr=3e-3, lr_final=3e-5, box=1.1, band=0.05, clip=0.25,
                        band_share=0.5, gate_rms=0.02, gate_max=0.1, ref_circumradius=0.0, seed=4):
        o = hlbm_train_opts(int(samples), int(holdout), int(iterations), int(batch), float(lr),
                            float(lr_final), float(box), float(band), float(clip), float(band_share),
                            float(gate_rms), float(gate_max), float(ref_circumradius), int(seed))
        r = hlbm_train_report()
        prm = np.ascontiguousarray(list(param) + [0.0] * (3 - len(param)), dtype=np.float64)
        _check(lib().hlbm_train_indicator(self._ctx, int(shape), prm.ctypes.data, ctypes.byref(o),
                                          ctypes.byref(r)))
        return {name: getattr(r, name) for name, _ in hlbm_train_report._fields_}

    def set_indicator(self, shape, mode):
        _check(lib().hlbm_set_indicator(self._ctx, int(shape), int(mode)))
