"""Metropolis chain driver: free run and replay of a logged run.  FP64.

Test infrastructure (see package docstring).

Section 2.2: at each step one particle is moved a small random distance; the
trial configuration is accepted when |Psi(R')|^2/|Psi(R)|^2 exceeds a uniform
draw on (0,1); a sweep moves every particle once.  Without the Jastrow factor
(ignored in the paper) the probability ratio is ratio^2 with ratio =
det(A')/det(A) (eq. (detRatioEq)).

Readings: particles are visited in order of their original id, p = g mod n for
the walker's g-th step; the test is strict, ratio^2 > u_acc; the move and the
acceptance draw come from ``rng.step_draws``.

Ratio modes: ``"lu"`` factors the current dense A at every step; ``"sm"`` is
the standard algorithm (explicit inverse, Sherman-Morrison on accept, refreshed
at every sweep boundary).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from .energy import kinetic_energy
from .geometry import orbital_values, propose, slater_dense
from .ratio import StandardAlgorithm, ratio_lu
from .rng import step_draws


@dataclasses.dataclass
class StepRecord:
    """One Metropolis step (Section 2.2): the walker's step counter g, the
    moved particle, its trial position, the ratio, the acceptance draw and the
    decision."""
    g: int
    particle: int
    new_pos: np.ndarray
    ratio: float
    u_acc: float
    accepted: bool


def free_run(system, pos0, seed: int, h: float, n_steps: int, start_step: int = 0,
             mode: str = "lu") -> (List[StepRecord], np.ndarray):
    """Metropolis steps start_step .. start_step + n_steps - 1 from pos0
    (Section 2.2): particle g mod n moves to a uniform trial point, the ratio
    det(A')/det(A) (eq. (detRatioEq)) comes from dense LU or the standard
    algorithm, and the move is accepted when ratio^2 exceeds the draw.
    Returns the records and the final positions."""
    n = system.n
    pos = np.array(pos0, dtype=np.float64, copy=True)
    A = slater_dense(pos, system)
    sm = StandardAlgorithm(A) if mode == "sm" else None
    out = []
    for g in range(start_step, start_step + n_steps):
        p = g % n
        if sm is not None and p == 0 and g != start_step:
            sm.refresh()
        u = step_draws(seed, g)
        rnew = propose(pos[p], u[:3], h, system.box)
        new_row = orbital_values(rnew, system)
        if sm is None:
            ratio, _ = ratio_lu(A, p, new_row)
        else:
            ratio = sm.ratio(p, new_row)
        acc = ratio * ratio > u[3]
        out.append(StepRecord(g, p, rnew, ratio, u[3], bool(acc)))
        if acc:
            if sm is not None:
                sm.accept(p, new_row, ratio)
            A[p] = new_row
            pos[p] = rnew
    return out, pos


def sweep_energies(system, pos0, seed: int, h: float, sweeps: int, start_step: int = 0,
                   mode: str = "sm"):
    """Free run of whole sweeps, sampling the kinetic energy per particle
    (eq. (energyEq)) at the end of every sweep (Section 4).  Returns the list
    of energies, the acceptance count and the final positions."""
    n = system.n
    pos = np.array(pos0, dtype=np.float64, copy=True)
    energies, accepted = [], 0
    for s in range(sweeps):
        recs, pos = free_run(system, pos, seed, h, n, start_step=start_step + s * n, mode=mode)
        accepted += sum(1 for r in recs if r.accepted)
        energies.append(kinetic_energy(pos, system))
    return energies, accepted, pos


def positions_after(pos0, log):
    """Positions after following a step log (records with particle, new_pos,
    accepted) from pos0: an accepted move replaces one particle's position
    (Section 2.2)."""
    pos = np.array(pos0, dtype=np.float64, copy=True)
    for rec in log:
        if rec.accepted:
            pos[int(rec.particle)] = np.asarray(rec.new_pos, dtype=np.float64)
    return pos


@dataclasses.dataclass
class ReplayReport:
    """What a replay found: per checked step |dln|ratio||, and the counts of
    trial positions, signs and decisions (Section 2.2's acceptance test) that
    differ from the log."""
    steps: int = 0
    max_dlog: float = 0.0
    dlogs: list = dataclasses.field(default_factory=list)
    pos_mismatch: int = 0
    sign_mismatch: int = 0
    decision_mismatch: int = 0
    decision_mismatch_outside_tol: int = 0
    oracle_ratios: list = dataclasses.field(default_factory=list)

    def summary(self) -> str:
        """Max and 99.9th percentile of |dln|ratio|| over the checked steps,
        and the decision mismatches (all, and those outside the tolerance)."""
        p999 = float(np.percentile(self.dlogs, 99.9)) if self.dlogs else 0.0
        return (f"{self.steps} steps: max dlog {self.max_dlog:.3e}, p99.9 {p999:.3e}; "
                f"decisions off {self.decision_mismatch} ({self.decision_mismatch_outside_tol} outside tol)")


def replay(system, pos0, seed: int, h: float, log, dec_tol: float = 1e-9,
           mode: str = "lu", check_every: int = 1) -> ReplayReport:
    """Follow a logged run (records with g, particle, new_pos, ratio, accepted),
    recomputing each move and ratio (Section 2.2, eq. (detRatioEq)); the logged
    decisions are followed, and a differing decision is classed by whether
    |ratio^2 - u| exceeds dec_tol (reading R6).

    ``check_every`` > 1 computes the oracle ratio only on every k-th step (in
    ``lu`` mode), replaying positions in between."""
    n = system.n
    pos = np.array(pos0, dtype=np.float64, copy=True)
    A = slater_dense(pos, system)
    sm = StandardAlgorithm(A) if mode == "sm" else None
    rep = ReplayReport()
    first = True
    for idx, rec in enumerate(log):
        g, p = int(rec.g), int(rec.particle)
        if sm is not None and p == 0 and not first:
            sm.refresh()
        first = False
        u = step_draws(seed, g)
        rnew = propose(pos[p], u[:3], h, system.box)
        if p != g % n or not np.array_equal(rnew, np.asarray(rec.new_pos)):
            rep.pos_mismatch += 1
        new_row = orbital_values(rnew, system)
        if sm is not None or idx % check_every == 0:
            if sm is None:
                ratio, _ = ratio_lu(A, p, new_row)
            else:
                ratio = sm.ratio(p, new_row)
            rep.steps += 1
            rep.oracle_ratios.append(ratio)
            if np.sign(ratio) != np.sign(rec.ratio):
                rep.sign_mismatch += 1
            dl = abs(np.log(abs(rec.ratio)) - np.log(abs(ratio))) if rec.ratio != 0 and ratio != 0 \
                else (0.0 if rec.ratio == ratio else np.inf)
            rep.dlogs.append(dl)
            rep.max_dlog = max(rep.max_dlog, dl)
            mine = ratio * ratio > u[3]
            if bool(mine) != bool(rec.accepted):
                rep.decision_mismatch += 1
                if abs(ratio * ratio - u[3]) > dec_tol:
                    rep.decision_mismatch_outside_tol += 1
        if rec.accepted:
            if sm is not None:
                sm.accept(p, new_row, ratio)
            A[p] = new_row
            pos[p] = rnew
    return rep
