"""CPU fp64 oracle of the parallel pulling protocol -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1105_4840_amd``) and never imports it.

* ``ppp_oracle.c``   -- Philox4x32-10, Box-Muller, potentials, integrators and
  the per-replica sample streams of every window (Sec. III(ii)).
* ``estimators.py``  -- Eqs. 9, 12, 13, 14, the combined estimate and its
  uncertainty (Sec. IV B, IV D), the JE variance formula, overlap diagnostics.
* ``appc.py``        -- work distributions from the xi distributions (App. C).
* ``quadrature.py``  -- exact restrained free energies by numerical quadrature
  and closed forms (the plain definition F(lambda,k) = -kT ln Z(lambda,k)).
* ``mlp.py``         -- fp64 reference of the 1-64-64-1 tanh surrogate with
  bf16 rounding emulation.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


class OracleProblem(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32),
        ("pot_kind", ctypes.c_int32),
        ("pot_a", ctypes.c_double), ("pot_b", ctypes.c_double), ("pot_kappa", ctypes.c_double),
        ("mobility", ctypes.c_double),
        ("integrator_1d", ctypes.c_int32),
        ("n_beads", ctypes.c_int32),
        ("k_bond", ctypes.c_double), ("r0", ctypes.c_double), ("k_angle", ctypes.c_double),
        ("lj_eps", ctypes.c_double), ("lj_sigma", ctypes.c_double), ("lj_rc", ctypes.c_double),
        ("rc_mode", ctypes.c_int32),
        ("mass", ctypes.c_double), ("gamma", ctypes.c_double),
        ("n_windows", ctypes.c_int32),
        ("lambda_", ctypes.POINTER(ctypes.c_double)),
        ("k", ctypes.c_double), ("kT", ctypes.c_double), ("dt", ctypes.c_double),
        ("n_steps", ctypes.c_int64), ("n_equil", ctypes.c_int64),
        ("sample_every", ctypes.c_int32),
        ("n_replicas", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("init_coords", ctypes.POINTER(ctypes.c_double)),
        ("xi_bound", ctypes.c_double),
        ("n_pull", ctypes.c_int64),
        ("sequential", ctypes.c_int32),
        ("free_ensemble", ctypes.c_int32),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(OracleProblem)
        L.oracle_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.oracle_normals4.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4 + [dp]
        L.oracle_normals6.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4 + [dp]
        L.oracle_chain_forces.argtypes = [pp, dp, ctypes.c_double, dp, dp]
        L.oracle_chain_forces.restype = ctypes.c_double
        L.oracle_pot1d.argtypes = [pp, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_pot1d.restype = ctypes.c_double
        L.oracle_default_helix.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.oracle_samples_per_replica.argtypes = [pp]
        L.oracle_samples_per_replica.restype = ctypes.c_int64
        L.oracle_run.argtypes = [pp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_trajectory.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp]
        _LIB = L
    return _LIB


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Problem:
    """Keeps the numpy buffers referenced by the ctypes struct alive."""

    def __init__(self, prob: dict):
        self.lam = np.ascontiguousarray(np.asarray(prob.get("lambda", [0.0]), dtype=np.float64))
        ic = prob.get("init_coords")
        self.init = None if ic is None else np.ascontiguousarray(np.asarray(ic, dtype=np.float64).ravel())
        model = 0 if prob["model"] == "1d" else 1
        self.s = OracleProblem(
            model=model,
            pot_kind=int(prob.get("pot_kind", 0)),
            pot_a=float(prob.get("pot_a", 5.0)), pot_b=float(prob.get("pot_b", 1.0)),
            pot_kappa=float(prob.get("pot_kappa", 1.0)),
            mobility=float(prob.get("mobility", 1.0)),
            integrator_1d=int(prob.get("integrator_1d", 0)),
            n_beads=int(prob.get("n_beads", 1)),
            k_bond=float(prob.get("k_bond", 100.0)), r0=float(prob.get("r0", 1.0)),
            k_angle=float(prob.get("k_angle", 5.0)),
            lj_eps=float(prob.get("lj_eps", 1.0)), lj_sigma=float(prob.get("lj_sigma", 1.0)),
            lj_rc=float(prob.get("lj_rc", 2.5)),
            rc_mode=int(prob.get("rc_mode", 0)),
            mass=float(prob.get("mass", 1.0)), gamma=float(prob.get("gamma", 1.0)),
            n_windows=len(self.lam),
            lambda_=_dp(self.lam),
            k=float(prob.get("k", 0.0)), kT=float(prob.get("kT", 1.0)), dt=float(prob.get("dt", 0.0)),
            n_steps=int(prob.get("n_steps", 0)), n_equil=int(prob.get("n_equil", 0)),
            sample_every=int(prob.get("sample_every", 1)),
            n_replicas=int(prob.get("n_replicas", 1)),
            seed=int(prob.get("seed", 0)),
            init_coords=None if self.init is None else _dp(self.init),
            xi_bound=float(prob.get("xi_bound", 1.0e4)),
            n_pull=int(prob.get("n_pull", 0)),
            sequential=1 if prob.get("sequential", False) else 0,
            free_ensemble=1 if prob.get("free_ensemble", False) else 0,
        )

    def ref(self):
        return ctypes.byref(self.s)


def philox(key, ctr):
    """Philox4x32-10 block for key (2 words) and counter (4 words)."""
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(k, c, o)
    return [int(x) for x in o]


def normals4(seed, c0, c1, c2, c3):
    z = np.zeros(4)
    lib().oracle_normals4(int(seed), c0, c1, c2, c3, _dp(z))
    return z


def normals6(seed, c0, c1, c2, c3):
    """Six normals of one block (the chain's noise: two beads per block)."""
    z = np.zeros(6)
    lib().oracle_normals6(int(seed), c0, c1, c2, c3, _dp(z))
    return z


def chain_forces(prob: dict, coords, lam):
    """Energy parts {bond, angle, lj, restraint}, total energy and forces."""
    P = _Problem(prob)
    r = np.ascontiguousarray(np.asarray(coords, dtype=np.float64).ravel())
    f = np.zeros_like(r)
    parts = np.zeros(4)
    e = lib().oracle_chain_forces(P.ref(), _dp(r), float(lam), _dp(f), _dp(parts))
    return e, parts, f.reshape(-1, 3)


def pot1d(prob: dict, x, lam):
    P = _Problem(prob)
    F = ctypes.c_double()
    e = lib().oracle_pot1d(P.ref(), float(x), float(lam), ctypes.byref(F))
    return e, F.value


def default_helix(n_beads, r0=1.0):
    r = np.zeros(3 * n_beads)
    lib().oracle_default_helix(int(n_beads), float(r0), _dp(r))
    return r.reshape(-1, 3)


def samples_per_replica(prob: dict) -> int:
    P = _Problem(prob)
    return int(lib().oracle_samples_per_replica(P.ref()))


def run(prob: dict, n_threads: int = 0):
    """Runs every replica of every window; returns (xi [W*R, S], n_kept [W*R], threads)."""
    P = _Problem(prob)
    S = int(lib().oracle_samples_per_replica(P.ref()))
    total = (len(P.lam) + (1 if prob.get("free_ensemble", False) else 0)) * int(prob["n_replicas"])
    xi = np.full((total, max(S, 1)), np.nan)
    kept = np.zeros(total, dtype=np.int64)
    used = lib().oracle_run(P.ref(), _dp(xi), kept.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            int(n_threads))
    return xi[:, :S], kept, int(used)


def trajectory(prob: dict, window: int, replica: int, n_steps: int):
    P = _Problem(prob)
    dof = 1 if prob["model"] == "1d" else 3 * int(prob["n_beads"])
    out = np.zeros((n_steps + 1) * dof)
    lib().oracle_trajectory(P.ref(), int(window), int(replica), int(n_steps), _dp(out))
    return out.reshape(n_steps + 1, dof)
