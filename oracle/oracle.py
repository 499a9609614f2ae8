"""ctypes binding of the plain FP64 CPU oracle (``hlbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It does not import
the HIP package and the HIP package never imports it.

Arrays follow the oracle's own storage: populations ``f[cell, i]`` (19 per
cell, this file's velocity order), scalar fields ``[cell]``, vector fields
``[3, cell]``, with ``cell = x + nx*(y + ny*z)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hlbm_oracle.c")
LIB = os.path.join(HERE, "libhlbm_oracle.so")

Q = 19


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over z-slabs)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
             SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class OCfg(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("bc", ctypes.c_int * 3), ("tau", ctypes.c_double),
                ("eps", ctypes.c_double), ("rho_f", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("af", ctypes.c_double * 3), ("coupling", ctypes.c_int)]


# the oracle's own particle record
OPART = np.dtype([("X", "<f8", 3), ("q", "<f8", 4), ("U", "<f8", 3), ("W", "<f8", 3),
                  ("m", "<f8"), ("V", "<f8"), ("I", "<f8", 3), ("prm", "<f8", 3),
                  ("shape", "<i4"), ("flags", "<i4")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(OCfg)
        vp = ctypes.c_void_p
        L.orc_tables.argtypes = [ctypes.POINTER(ctypes.c_int), dp, ctypes.POINTER(ctypes.c_int)]
        L.orc_feq.argtypes = [ctypes.c_double, dp, dp]
        L.orc_sdf.argtypes = [ctypes.c_int, dp, dp]
        L.orc_sdf.restype = ctypes.c_double
        L.orc_set_mesh.argtypes = [dp, ctypes.c_int]
        L.orc_set_contact.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_contact_forces.argtypes = [cp, ctypes.c_int, vp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, dp, dp]
        L.orc_set_contact_nodes.argtypes = [ctypes.c_int]
        L.orc_circumradius.argtypes = [ctypes.c_int, dp]
        L.orc_circumradius.restype = ctypes.c_double
        L.orc_indicator.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_indicator.restype = ctypes.c_double
        L.orc_equilibrium_field.argtypes = [cp, vp, vp, dp]
        L.orc_moments.argtypes = [cp, dp, dp, dp]
        L.orc_collide_cell.argtypes = [cp, dp, ctypes.c_double, dp, dp]
        L.orc_collide_cell_psm.argtypes = [cp, dp, ctypes.c_double, dp, dp]
        L.orc_psm_weight.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_psm_weight.restype = ctypes.c_double
        L.orc_collide.argtypes = [cp, dp, dp, dp, dp]
        L.orc_stream.argtypes = [cp, dp, dp]
        L.orc_mea.argtypes = [cp, ctypes.c_int, vp, dp, dp, dp]
        L.orc_apply_eom.argtypes = [cp, ctypes.c_int, vp, dp, dp]
        L.orc_coupling.argtypes = [cp, ctypes.c_int, vp, dp, dp]
        L.orc_run.argtypes = [cp, ctypes.c_int, vp, dp, ctypes.c_int, vp, vp]
        L.orc_run.restype = ctypes.c_int
        L.orc_fields.argtypes = [cp, ctypes.c_int, vp, dp, dp, dp, dp, vp]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """A lattice configuration plus the oracle's passes over numpy arrays."""

    def __init__(self, n, bc=(0, 0, 0), tau=0.8, eps=0.5, rho_f=1.0, gravity=(0.0, 0.0, 0.0),
                 fluid_accel=(0.0, 0.0, 0.0), contact=None, coupling="hlbm"):
        # coupling: "hlbm" (exact-difference source) or "psm" (partially
        # saturated collision); the particle force is the MEA's in both
        # contact: None, or (range zeta, stiffness k, wall stiffness k_w) of the
        # sphere repulsion added to the equations of motion
        self.contact = tuple(float(v) for v in contact) if contact else (0.0, 0.0, 0.0)
        self.n = tuple(int(v) for v in n)
        self.bc = tuple(int(v) for v in bc)
        self.cfg = OCfg((ctypes.c_int * 3)(*self.n), (ctypes.c_int * 3)(*self.bc), float(tau),
                        float(eps), float(rho_f), (ctypes.c_double * 3)(*gravity),
                        (ctypes.c_double * 3)(*fluid_accel), {"hlbm": 0, "psm": 1}[coupling])
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.tau = float(tau)
        self.eps = float(eps)

    def set_fluid_accel(self, accel):
        """Replace the fluid body acceleration for the following runs."""
        self.cfg.af = (ctypes.c_double * 3)(*[float(v) for v in accel])

    # ---- tables ---------------------------------------------------------
    @staticmethod
    def tables():
        c = (ctypes.c_int * (3 * Q))()
        w = np.zeros(Q)
        opp = (ctypes.c_int * Q)()
        lib().orc_tables(c, _dp(w), opp)
        return np.array(list(c), dtype=np.int64).reshape(Q, 3), w, np.array(list(opp))

    # ---- pointwise ------------------------------------------------------
    @staticmethod
    def feq(rho, u):
        out = np.zeros(Q)
        uu = np.ascontiguousarray(u, dtype=np.float64)
        lib().orc_feq(float(rho), _dp(uu), _dp(out))
        return out

    @staticmethod
    def sdf(shape, prm, p):
        prm = np.ascontiguousarray(prm, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        return lib().orc_sdf(int(shape), _dp(prm), _dp(p))

    @staticmethod
    def circumradius(shape, prm):
        prm = np.ascontiguousarray(prm, dtype=np.float64)
        return lib().orc_circumradius(int(shape), _dp(prm))

    def indicator(self, d):
        return lib().orc_indicator(float(d), self.eps)

    def collide_cell(self, f, B=0.0, us=(0.0, 0.0, 0.0)):
        f = np.ascontiguousarray(f, dtype=np.float64)
        us = np.ascontiguousarray(us, dtype=np.float64)
        out = np.zeros(Q)
        fn = lib().orc_collide_cell_psm if self.cfg.coupling == 1 else lib().orc_collide_cell
        fn(ctypes.byref(self.cfg), _dp(f), float(B), _dp(us), _dp(out))
        return out

    def psm_weight(self, B):
        return lib().orc_psm_weight(float(B), self.tau)

    # ---- fields ---------------------------------------------------------
    def equilibrium(self, rho=None, u=None):
        f = np.zeros((self.N, Q))
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(3, -1)
        lib().orc_equilibrium_field(ctypes.byref(self.cfg),
                                    None if r is None else r.ctypes.data,
                                    None if v is None else v.ctypes.data, _dp(f))
        return f

    def moments(self, f):
        rho = np.zeros(self.N)
        u = np.zeros((3, self.N))
        lib().orc_moments(ctypes.byref(self.cfg), _dp(f), _dp(rho), _dp(u))
        return rho, u

    def collide(self, f, B, us):
        out = np.zeros_like(f)
        lib().orc_collide(ctypes.byref(self.cfg), _dp(f), _dp(np.ascontiguousarray(B)),
                          _dp(np.ascontiguousarray(us)), _dp(out))
        return out

    def stream(self, fs):
        out = np.zeros_like(fs)
        lib().orc_stream(ctypes.byref(self.cfg), _dp(fs), _dp(out))
        return out

    # ---- particles ------------------------------------------------------
    # the closed triangle mesh of shape 3 particles (one per process): unit
    # scale, and its largest vertex radius
    mesh_rc = 0.0

    @classmethod
    def set_mesh(cls, vertices, triangles):
        """vertices [nv, 3] (body frame, unit scale), triangles [nt, 3] vertex
        indices, counter-clockwise seen from outside."""
        v = np.asarray(vertices, dtype=np.float64)
        tri = np.ascontiguousarray(v[np.asarray(triangles)], dtype=np.float64)  # [nt, 3, 3]
        lib().orc_set_mesh(_dp(tri), len(tri))
        cls.mesh_rc = float(np.sqrt((tri ** 2).sum(axis=2)).max())

    def to_parts(self, particles) -> np.ndarray:
        """Copy a record array with fields pos/quat/vel/omega/mass/volume/
        inertia/param/shape into the oracle's own record layout."""
        P = np.zeros(len(particles), dtype=OPART)
        if len(particles):
            P["X"] = particles["pos"]
            P["q"] = particles["quat"]
            P["U"] = particles["vel"]
            P["W"] = particles["omega"]
            P["m"] = particles["mass"]
            P["V"] = particles["volume"]
            P["I"] = particles["inertia"]
            P["prm"] = particles["param"]
            P["shape"] = particles["shape"]
            mesh = P["shape"] == 3
            if np.any(mesh):  # circumradius of a mesh particle: scale x largest vertex radius
                P["prm"][mesh, 1] = P["prm"][mesh, 0] * self.mesh_rc
        self._check_parts(P)
        return P

    def _check_parts(self, P):
        """Every cell the passes visit for a particle (centre within the
        circumradius + max(eps/2, 1)) must be reached once, with an unambiguous
        minimum image: that reach must stay below half of a periodic extent."""
        for p in P:
            R = self.circumradius(int(p["shape"]), p["prm"]) + max(0.5 * self.eps, 1.0)
            for k in range(3):
                if self.bc[k] == 0 and 2 * R >= self.n[k]:
                    raise ValueError("particle reach exceeds half the periodic box")

    def mea(self, P, f):
        F = np.zeros((len(P), 3))
        T = np.zeros((len(P), 3))
        lib().orc_mea(ctypes.byref(self.cfg), len(P), P.ctypes.data if len(P) else None, _dp(f),
                      _dp(F), _dp(T))
        return F, T

    def apply_eom(self, P, F, T):
        F = np.ascontiguousarray(F, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64)
        lib().orc_apply_eom(ctypes.byref(self.cfg), len(P), P.ctypes.data if len(P) else None,
                            _dp(F), _dp(T))

    def coupling(self, P):
        B = np.zeros(self.N)
        us = np.zeros((3, self.N))
        lib().orc_coupling(ctypes.byref(self.cfg), len(P), P.ctypes.data if len(P) else None,
                           _dp(B), _dp(us))
        return B, us

    def run(self, P, f, nsteps):
        """Advance f and P in place by nsteps; returns the last MEA force/torque."""
        F = np.zeros((max(len(P), 1), 3))
        T = np.zeros((max(len(P), 1), 3))
        lib().orc_set_contact(*self.contact)
        lib().orc_run(ctypes.byref(self.cfg), len(P), P.ctypes.data if len(P) else None, _dp(f),
                      int(nsteps), F.ctypes.data, T.ctypes.data)
        return F[:len(P)], T[:len(P)]

    def contact_forces(self, P, contact=None, torque=False):
        """Contact forces [np, 3] on the state P (the repulsion the equations
        of motion add when contact is set); with torque, (forces, torques)."""
        rng, k, kw = (float(v) for v in (contact or self.contact))
        Fc = np.zeros((max(len(P), 1), 3))
        Tc = np.zeros((max(len(P), 1), 3))
        lib().orc_contact_forces(ctypes.byref(self.cfg), len(P), P.ctypes.data if len(P) else None, rng, k, kw,
                                 _dp(Fc), _dp(Tc))
        return (Fc[:len(P)], Tc[:len(P)]) if torque else Fc[:len(P)]

    @staticmethod
    def set_contact_nodes(M):
        """Surface nodes per particle of the non-spherical contact (1024)."""
        lib().orc_set_contact_nodes(int(M))

    def fields(self, P, f):
        rho = np.zeros(self.N)
        u = np.zeros((3, self.N))
        up = np.zeros((3, self.N))
        B = np.zeros(self.N)
        lib().orc_fields(ctypes.byref(self.cfg), len(P), P.ctypes.data if len(P) else None, _dp(f),
                         _dp(rho), _dp(u), _dp(up), B.ctypes.data)
        return rho, u, up, B

    @staticmethod
    def num_threads():
        return lib().orc_num_threads()
