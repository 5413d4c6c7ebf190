"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's checks.

This module holds parameter sets and random-number-driven input generators
only: none of the protocol's arithmetic.  The workloads stand in for the
paper's deca-alanine runs (Sec. IV: 21 windows, one shared start state,
independent windows): a one-particle double well and bead-spring chains whose
end-to-end distance plays the role of the pulled end's position.

Problems are plain dicts; both the GPU binding and the oracle read the same
keys.
"""
import numpy as np


def _lin(a, b, n):
    return [float(x) for x in np.linspace(a, b, n)]


def _hist_spec(lo, hi, nbins=4096):
    return {"xi_min": float(lo), "xi_bin": float(hi - lo) / nbins, "xi_nbins": int(nbins)}


def chain_forcefield(n_beads):
    """Bead-spring chain: harmonic bonds k_b = 100, r0 = 1; cosine angles k_theta = 5;
    Lennard-Jones eps = sigma = 1, cutoff 2.5 sigma, pairs |i-j| > 2; bead 0 fixed;
    unit mass; BAOAB with gamma = 1, dt = 0.005, kT = 1."""
    return {"model": "chain", "n_beads": int(n_beads), "k_bond": 100.0, "r0": 1.0, "k_angle": 5.0,
            "lj_eps": 1.0, "lj_sigma": 1.0, "lj_rc": 2.5, "rc_mode": 0, "mass": 1.0, "gamma": 1.0,
            "kT": 1.0, "dt": 0.005}


def config_1d(n_replicas=256, n_steps=20000, n_windows=21, seed=0, precision="fp64"):
    """One particle, U(x) = 5 (x^2 - 1)^2 kT, kT = 1, k = 50, 21 windows in [-1.5, 1.5],
    overdamped Langevin dt = 1e-3 started at x0 = lambda_1."""
    p = {"name": "1d-double-well", "model": "1d", "pot_kind": 0, "pot_a": 5.0, "pot_b": 1.0,
         "pot_kappa": 0.0, "mobility": 1.0, "integrator_1d": 0,
         "lambda": _lin(-1.5, 1.5, n_windows), "k": 50.0, "kT": 1.0, "dt": 1e-3,
         "n_steps": int(n_steps), "n_equil": int(n_steps) // 10, "sample_every": 10,
         "n_replicas": int(n_replicas), "seed": int(seed), "init_coords": None,
         "n_blocks": 32, "w_bin": 0.01, "w_half_bins": 15000, "precision": precision,
         "xi_bound": 1.0e4}
    p.update(_hist_spec(-2.5, 2.5))
    return p


def config_harmonic_1d(kappa=4.0, k=20.0, n_replicas=256, n_steps=20000, seed=1, precision="fp64"):
    """One particle in kappa/2 x^2 with the restraint: an exactly Gaussian xi (closed form)."""
    p = config_1d(n_replicas=n_replicas, n_steps=n_steps, seed=seed, precision=precision)
    p.update({"name": "1d-harmonic", "pot_kind": 1, "pot_kappa": float(kappa), "k": float(k),
              "lambda": _lin(-1.0, 1.0, 11)})
    p["init_coords"] = [-1.0]
    return p


def config_chain10(n_replicas=1024, n_steps=40000, seed=0, precision="fp32"):
    """10-bead chain, restraint k = 20 on the end-to-end distance, 21 windows in [1.5, 8.5]."""
    p = chain_forcefield(10)
    p.update({"name": "chain10", "lambda": _lin(1.5, 8.5, 21), "k": 20.0,
              "n_steps": int(n_steps), "n_equil": int(n_steps) // 10, "sample_every": 10,
              "n_replicas": int(n_replicas), "seed": int(seed), "init_coords": None,
              "n_blocks": 32, "w_bin": 0.01, "w_half_bins": 15000, "precision": precision,
              "xi_bound": 1.0e4})
    p.update(_hist_spec(0.0, 11.0))
    return p


def config_chain32(n_replicas=4096, n_steps=23251, n_windows=21, seed=0, precision="fp32",
                   lam=None):
    """32-bead chain, k = 20, windows in [3, 28] (uniform: 21 windows)."""
    p = chain_forcefield(32)
    p.update({"name": "chain32", "lambda": list(lam) if lam is not None else _lin(3.0, 28.0, n_windows),
              "k": 20.0, "n_steps": int(n_steps), "n_equil": int(n_steps) // 10, "sample_every": 10,
              "n_replicas": int(n_replicas), "seed": int(seed), "init_coords": None,
              "n_blocks": 32, "w_bin": 0.01, "w_half_bins": 45000, "precision": precision,
              "xi_bound": 1.0e4})
    p.update(_hist_spec(0.0, 33.0))
    return p


def config_chain256(n_replicas=4096, n_steps=200000, seed=0, precision="fp32"):
    """256-bead chain, k = 20, 41 windows in [10, 200], all Lennard-Jones pairs evaluated.
    The windows lie up to 90 length units from the shared start state, so the
    restraint centre is pulled there linearly over the first 5% of the steps."""
    p = chain_forcefield(256)
    p.update({"name": "chain256", "lambda": _lin(10.0, 200.0, 41), "k": 20.0,
              "n_steps": int(n_steps), "n_equil": int(n_steps) // 10, "sample_every": 10,
              "n_pull": int(n_steps) // 20,
              "n_replicas": int(n_replicas), "seed": int(seed), "init_coords": None,
              "n_blocks": 32, "w_bin": 0.05, "w_half_bins": 45000, "precision": precision,
              "xi_bound": 1.0e4})
    p.update(_hist_spec(0.0, 256.0, 8192))
    return p


def config_chain_small(n_beads, n_replicas=64, n_steps=4000, n_windows=6, seed=3, precision="fp64"):
    """Small chain problems for parity tests (several tiles and a ragged tail); the
    windows bracket the end-to-end distance of the helical start state (about
    0.395 (N-1)), so the relaxation is gentle."""
    p = chain_forcefield(n_beads)
    lo = 0.3 * (n_beads - 1) + 0.5
    top = 0.5 * (n_beads - 1) + 1.5
    p.update({"name": f"chain{n_beads}-small", "lambda": _lin(lo, top, n_windows), "k": 20.0,
              "n_steps": int(n_steps), "n_equil": int(n_steps) // 10, "sample_every": 10,
              "n_replicas": int(n_replicas), "seed": int(seed), "init_coords": None,
              "n_blocks": 8, "w_bin": 0.01, "w_half_bins": 6000, "precision": precision,
              "xi_bound": 1.0e4})
    p.update(_hist_spec(0.0, top + 3.0, 1024))
    return p


def batched_instances(n_chains=64, seed=0):
    """Uneven batch: chain lengths U{8..128}, windows U{11..41}, replicas per window in
    {64,128,256,512,1024}, steps log-uniform in [5e3, 1e5], lambda in
    [0.15 (N-1), 0.85 (N-1)], k = 20, one seed per chain."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_chains):
        n = int(rng.integers(8, 129))
        s = int(rng.integers(11, 42))
        R = int(rng.choice([64, 128, 256, 512, 1024]))
        steps = int(round(np.exp(rng.uniform(np.log(5e3), np.log(1e5)))))
        p = chain_forcefield(n)
        lo, hi = 0.15 * (n - 1), 0.85 * (n - 1)
        p.update({"name": f"batch{c}", "lambda": _lin(lo, hi, s), "k": 20.0,
                  "n_steps": steps, "n_equil": steps // 10, "sample_every": 10,
                  "n_pull": steps // 20,
                  "n_replicas": R, "seed": 1000 + c, "init_coords": None,
                  "n_blocks": 32, "w_bin": 0.01, "w_half_bins": 15000, "precision": "fp32",
                  "xi_bound": 1.0e4})
        p.update(_hist_spec(0.0, float(n), 4096))
        out.append(p)
    return out


def random_chain_coords(n_beads, n_conf, seed=0, jitter=0.15):
    """Random chain conformations near unit bonds, bead 0 at the origin: a
    persistent random walk grown bead by bead, each new bead redrawn until it
    is at least 0.8 from every earlier bead three or more positions back."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_conf):
        r = np.zeros((n_beads, 3))
        d = rng.normal(size=3); d /= np.linalg.norm(d)
        for i in range(1, n_beads):
            for _attempt in range(1000):
                e = d + 0.9 * rng.normal(size=3); e /= np.linalg.norm(e)
                cand = r[i - 1] + e * (1.0 + jitter * rng.normal())
                if i < 3 or np.min(np.linalg.norm(r[:i - 2] - cand, axis=1)) >= 0.8:
                    break
            d = e
            r[i] = cand
        out.append(r)
    return np.array(out)
