"""Periodic hindered settling (Sec. 5) on the HLBM library.

Spheres of diameter D = N cells settle in a fully periodic cube of edge 12 D.
The set-up is fixed by the Archimedes number Ar = g D^3 (rho_p/rho_f - 1) / nu^2
and the density ratio (Sec. 5.1: Ar = 1500, ratio 1.3, tau = 0.55).  The
reference velocity u* of a single sphere comes from the force balance with the
Schiller-Naumann drag coefficient.  The mean settling velocity is compared with
the power law u/u* = (1 - phi)^n using the Richardson-Zaki and
Garside-Al-Dibouni expansion indices, and with the Barnea-Mizrahi form
(Sec. 5, power-law and expansion-index equations).

As in Sec. 5.1, the fluid outside the particles is driven against the settling
by a body acceleration that keeps the net volume flux at zero.  The paper
derives the pressure gradient from the Ergun equation at the current settling
velocity.  Here a proportional-integral controller on the measured volume flux
sets it, starting from the static balance of the particles' submerged weight.
Either way the flux is held at zero.  The mean settling velocity is taken in
that frame as (1 - phi) (<U_p> - <u_f>), with <u_f> the mean velocity of the
pure-fluid cells.  This form does not depend on the frame, so any flux left
over by the controller does not bias it.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import hlbm as H
from . import workloads as W


def reynolds_schiller_naumann(Ar: float) -> float:
    """Terminal Reynolds number of a single sphere: with
    u*^2 = 4 g D (rho_p/rho_f - 1) / (3 C_d) and Re = u* D / nu, the balance
    reads (3/4) C_d Re^2 = Ar, and with C_d = 24/Re (1 + 0.15 Re^0.687)
    (Schiller-Naumann, Re < 800): 18 Re (1 + 0.15 Re^0.687) = Ar.  Solved by
    bisection (the left side increases with Re)."""
    lo, hi = 0.0, 1e4
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if 18.0 * mid * (1.0 + 0.15 * mid ** 0.687) < Ar:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def n_richardson_zaki(Re: float) -> float:
    """Richardson-Zaki expansion index (piecewise in Re)."""
    if Re < 0.2:
        return 4.65
    if Re < 1.0:
        return 4.35 * Re ** -0.03
    if Re < 500.0:
        return 4.45 * Re ** -0.1
    return 2.39


def n_garside_al_dibouni(Re: float) -> float:
    """Garside-Al-Dibouni expansion index."""
    r = Re ** 0.9
    return (5.1 + 0.27 * r) / (1.0 + 0.1 * r)


def barnea_mizrahi(phi: float) -> float:
    """Barnea-Mizrahi mean settling velocity over u* (independent of Re)."""
    return (1.0 - phi) / ((1.0 + phi ** (1.0 / 3.0)) * math.exp(5.0 * phi / (3.0 * (1.0 - phi))))


def power_law(phi: float, n: float) -> float:
    return (1.0 - phi) ** n


def particle_count(phi: float, box_diameters: float = 12.0) -> int:
    """Smallest number of spheres whose volume fraction in a cube of edge
    box_diameters * D reaches phi."""
    return math.ceil(phi * box_diameters ** 3 / (math.pi / 6.0))


def setup(Ar=1500.0, ratio=1.3, tau=0.55, N=12):
    """Lattice units of the set-up: nu from tau, g from Ar, the Stokes
    velocity (which defines t* = D / u_St), Re and u* from Schiller-Naumann."""
    nu = (tau - 0.5) / 3.0
    g = Ar * nu * nu / (N ** 3 * (ratio - 1.0))
    u_st = g * N * N * (ratio - 1.0) / (18.0 * nu)
    Re = reynolds_schiller_naumann(Ar)
    return dict(nu=nu, g=g, u_st=u_st, t_star=N / u_st, Re=Re, u_star=Re * nu / N, N=N, Ar=Ar,
                ratio=ratio, tau=tau)


def place_spheres(phi, N, seed, gap):
    """Random sequential addition of equal spheres in the periodic cube."""
    L = 12 * N
    count = particle_count(phi)
    rng = np.random.default_rng(seed)
    pos = W.rsa_positions(rng, np.full(count, N / 2.0), (L, L, L), (0, 0, 0), gap=gap)
    return L, pos


def run_periodic(phi, N=12, Ar=1500.0, ratio=1.3, tau=0.55, t_total=300.0, t_avg=30.0, precision="fp32",
                 seed=7, gap=1.0, control_every=20, sample_every=None, log=None, contact=None):
    """Settle the suspension for t_total t* and average the settling velocity
    from t_avg t* on.  Returns the set-up, u_bar / u*, its standard error (from
    the means of 10 consecutive batches of samples, which are far less
    correlated than single samples), the three correlations, the residual
    volume flux and the wall time.

    contact = (range, factor) turns on the contact repulsion of the library
    (hlbm_set_contact) with that range in cells and a stiffness of `factor`
    times one sphere's submerged weight (the force at touching)."""
    import torch
    s = setup(Ar, ratio, tau, N)
    L, pos = place_spheres(phi, N, seed, gap)
    recs = np.array([W.make_particle(W.SPHERE, (N / 2.0,), p, density_ratio=ratio) for p in pos])
    count = len(recs)
    phi_v = count * math.pi * N ** 3 / 6.0 / L ** 3
    g = s["g"]
    # static balance: the fluid outside the particles carries the particles'
    # submerged weight
    a0 = (ratio - 1.0) * g * phi_v / (1.0 - phi_v)
    sim = H.Simulation((L, L, L), (0, 0, 0), tau, precision, max_particles=count, gravity=(0.0, 0.0, -g),
                       fluid_accel=(0.0, 0.0, a0))
    sim.set_particles(recs)
    if contact:
        weight = (ratio - 1.0) * g * math.pi * N ** 3 / 6.0
        sim.set_contact(float(contact[0]), float(contact[1]) * weight, 0.0)
    nsteps = int(round(t_total * s["t_star"]))
    n_avg = int(round(t_avg * s["t_star"]))
    sample_every = sample_every or max(control_every, int(round(s["t_star"] / 2)) // control_every * control_every)
    # PI control of the volume flux J (critically damped at w = 1 / (5 t*))
    w = 1.0 / (5.0 * s["t_star"])
    kp, ki = 2.0 * w, w * w
    integ, af = 0.0, a0
    vals, flux = [], []
    t0 = time.perf_counter()
    done = 0
    while done < nsteps:
        k = min(control_every, nsteps - done)
        sim.step(k)
        done += k
        # volume flux (particle cells move with the particles) and the mean
        # velocity of the pure-fluid cells, both reduced by the library
        mean_all, mean_fluid, _ = sim.get_mean_velocity()
        J = float(mean_all[2])
        integ += J * k
        af = a0 - kp * J - ki * integ
        sim.set_fluid_accel((0.0, 0.0, af))
        if done >= n_avg and done % sample_every == 0:
            uf = float(mean_fluid[2])
            _, _, st = sim.get_forces()
            up = float(np.mean(st["vel"][:, 2]))
            vals.append(-(1.0 - phi_v) * (up - uf))
            flux.append(J)
            if log and len(vals) % 50 == 0:
                log(f"  phi {phi_v:.3f}: step {done}/{nsteps}, u_bar/u* so far {np.mean(vals) / s['u_star']:.4f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    nacc = len(vals)
    u_bar = float(np.mean(vals)) if vals else 0.0
    batches = np.array_split(np.asarray(vals), 10) if nacc >= 20 else []
    se = float(np.std([b.mean() for b in batches], ddof=1) / math.sqrt(len(batches))) if batches else float("nan")
    Re = s["Re"]
    return dict(phi=phi_v, count=count, steps=nsteps, samples=nacc, seconds=wall, u_star=s["u_star"],
                ratio=u_bar / s["u_star"], ratio_se=se / s["u_star"], rz=power_law(phi_v, n_richardson_zaki(Re)),
                gad=power_law(phi_v, n_garside_al_dibouni(Re)), bm=barnea_mizrahi(phi_v), Re=Re,
                mean_flux=float(np.mean(flux)) if flux else 0.0, final_accel=af, static_accel=a0)


def main(argv=None):
    """python -m paper_2312_14172_amd.settling --phi 0.05 0.1 --N 12: one JSON
    line per volume fraction."""
    import argparse
    import json
    import torch
    ap = argparse.ArgumentParser(description="periodic hindered settling (Ar, density ratio, tau as in Sec. 5.1)")
    ap.add_argument("--phi", type=float, nargs="+", default=[0.05, 0.1, 0.2, 0.3])
    ap.add_argument("--N", type=int, default=12, help="cells per sphere diameter")
    ap.add_argument("--t-total", type=float, default=300.0)
    ap.add_argument("--t-avg", type=float, default=30.0)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--gap", type=float, default=None, help="RSA surface gap (default 1, 0.2 from phi 0.25)")
    ap.add_argument("--contact", type=float, nargs=2, default=None, metavar=("RANGE", "FACTOR"),
                    help="sphere repulsion: range in cells, stiffness in submerged weights")
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    H.lib()
    for phi in a.phi:
        gap = a.gap if a.gap is not None else (1.0 if phi < 0.25 else 0.2)
        r = run_periodic(phi, N=a.N, t_total=a.t_total, t_avg=a.t_avg, precision=a.precision, seed=a.seed,
                         gap=gap, log=lambda m: print(m, flush=True), contact=a.contact)
        r["N"] = a.N
        r["contact"] = a.contact
        print(json.dumps({k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}), flush=True)


if __name__ == "__main__":
    main()
