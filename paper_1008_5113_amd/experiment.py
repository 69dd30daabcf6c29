"""The paper's own experiment (Section 4) on the GPU.

n = 2K^3 electrons in Gaussian orbitals exp(-k|d|^2), k = 1, on a b.c.c.
lattice of K^3 cubes of side 2.031; entries below 1e-5 of the largest dropped;
ILUTP droptol 0.01 (scaled by each row's mean magnitude, as SPARSKIT's ILUTP
does) with column pivoting at permtol 0.05; full GMRES with rtol 1e-6 and at most 40
iterations; reorder when N > 100 or the iterations reach four times their
average; 120 sweeps with the first 20 discarded; the kinetic energy per
particle (eq. (energyEq)) sampled at the end of every sweep, here through the
same preconditioned solver.  Many walkers run side by side (one workgroup
each), so the energy's error bar comes from the spread of the walkers' means.

Reported beside the paper's Table "cost" and Table "energy" figures: the
acceptance ratio, the average GMRES iterations per solve (k_1), nonzeros per row
of A (k_2) and of L + U (alpha k_2), reorders per sweep (k_5) and the energy.

    python -m paper_1008_5113_amd.experiment --sizes 686,1024 --walkers 64
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

import workloads as wl

from .vmcdet import FLAG_ACCEPTED, FLAG_REORDERED, Context

# Section 4, Table "cost" (k_1, k_2, alpha k_2, k_5) and Table "energy" (the
# sparse algorithm's kinetic energy and its standard deviation), by n.
PAPER_TABLES = {
    686: dict(iters=8.91, nnz_a=42.38, nnz_lu=55.04, reorders=0.65, energy=2.0984, energy_sd=0.0075, acc=0.5879),
    1024: dict(iters=9.34, nnz_a=42.38, nnz_lu=54.48, reorders=1.03, energy=2.1074, energy_sd=0.0077, acc=0.5880),
    1458: dict(iters=9.53, nnz_a=42.39, nnz_lu=54.33, reorders=1.19, energy=2.1107, energy_sd=0.0040, acc=0.5887),
    2000: dict(iters=9.59, nnz_a=42.38, nnz_lu=53.61, reorders=1.73, energy=2.1040, energy_sd=0.0034, acc=0.5880),
    2662: dict(iters=9.83, nnz_a=42.37, nnz_lu=53.27, reorders=2.23, energy=2.1010, energy_sd=0.0023, acc=0.5881),
    3456: dict(iters=10.20, nnz_a=42.37, nnz_lu=53.28, reorders=2.63, energy=2.0999, energy_sd=0.0045, acc=0.5898),
    4394: dict(iters=10.22, nnz_a=42.37, nnz_lu=53.28, reorders=2.73, energy=2.1049, energy_sd=0.0033, acc=0.5878),
    5488: dict(iters=10.10, nnz_a=42.37, nnz_lu=53.01, reorders=3.12, energy=2.1010, energy_sd=0.0034, acc=0.5883),
}


PHASES = ("prepare", "lsolve", "usolve", "updates", "spmv", "ortho", "solution", "resid64", "accept",
          "refactor", "reorder")


def run(K: int, n_walkers: int = 64, sweeps: int = 120, discard: int = 20, keep_walker0: int = 0,
        step: float = 0.55, permtol: float = 0.05, autotune: bool = True, progress=None,
        chunks: int = 1, note=None) -> dict:
    """Run the experiment for n = 2K^3; `chunks` launches per sweep (one by
    default).  With autotune the refactor period follows the cost balance of
    Section 3.2 (measured during one extra sweep before the first);
    keep_walker0 > 0 also returns walker 0's step records of the first
    keep_walker0 sweeps; progress(s) is called after every sweep, note(text)
    after the set-up stages and after every launch."""
    inst = wl.paper_bcc(K=K, n_walkers=n_walkers, step=step, sweeps=sweeps, permtol=permtol)
    n = inst.systems[0].n
    if not 1 <= chunks <= n:
        raise ValueError("chunks must lie in [1, n]")
    say = note or (lambda text: None)
    kw = {"m_max": 200} if autotune else {}
    ctx = Context.from_instance(inst, **kw)
    try:
        t = time.perf_counter()
        ctx.ilutp(reorder=True)
        ctx.sync()
        say(f"n={n}: reorder + ILUTP of {n_walkers} walkers {time.perf_counter() - t:.1f}s")
        if autotune:
            t = time.perf_counter()
            ctx.autotune(trial_steps=n)
            say(f"n={n}: autotune (one sweep) {time.perf_counter() - t:.1f}s")
        pos_start = ctx.state(0)["pos"] if keep_walker0 else None
        st0 = ctx.stats()
        energies = np.zeros((n_walkers, sweeps))
        acc = iters = reorders = steps = 0
        kept = []
        t0 = time.perf_counter()
        bounds = [n * c // chunks for c in range(chunks + 1)]
        for s in range(sweeps):
            parts = []
            for c in range(chunks):
                e, part = ctx.run_steps_energy(bounds[c + 1] - bounds[c], energy_cap=1, log=True)
                parts.append(part)
                if chunks > 1:
                    say(f"sweep {s + 1}: launch {c + 1}/{chunks}")
            # the energy is sampled once, at the sweep end (the last launch)
            energies[:, s] = e[:, 0]
            log = np.concatenate(parts, axis=1) if chunks > 1 else parts[0]
            flags = log["flags"]
            acc += int(np.count_nonzero(flags & FLAG_ACCEPTED))
            reorders += int(np.count_nonzero(flags & FLAG_REORDERED))
            iters += int(log["iters"].sum())
            steps += flags.size
            if s < keep_walker0:
                kept.append(log[0].copy())
            if progress:
                progress(s)
        elapsed = time.perf_counter() - t0
        st1 = ctx.stats()
        nnz_a = nnz_lu = 0.0
        for w in range(min(n_walkers, 8)):
            f = ctx.state(w, factors=True)
            nnz_a += float(np.sum(f["a_len"])) / n
            nnz_lu += float(np.sum(f["l_len"]) + np.sum(f["u_len"]) + n) / n
        nw = min(n_walkers, 8)
        status = [s["status"] for s in st1]
    finally:
        ctx.close()
    means = energies[:, discard:].mean(axis=1)
    out = dict(
        n=n, walkers=n_walkers, sweeps=sweeps, discard=discard, step=step, permtol=permtol,
        acceptance=acc / steps,
        iters_per_solve=iters / steps,
        nnz_a=nnz_a / nw,
        nnz_lu=nnz_lu / nw,
        reorders_per_sweep=reorders / (n_walkers * sweeps),
        reorders_per_sweep_all=sum(b["reorders"] - a["reorders"] for a, b in zip(st0, st1)) / (n_walkers * sweeps),
        energy=float(means.mean()),
        energy_sd=float(means.std(ddof=1) / np.sqrt(n_walkers)) if n_walkers > 1 else float("nan"),
        seconds_per_sweep=elapsed / sweeps,
        autotune=autotune,
        phase_fraction=_phase_fractions(st0, st1),
        status_ok=all(s == 0 for s in status),
        paper=PAPER_TABLES.get(n),
    )
    if keep_walker0:
        out["walker0_log"] = np.concatenate(kept)
        out["walker0"] = inst.walkers[0]
        out["walker0_pos"] = pos_start   # positions where the kept records start
        out["system"] = inst.systems[0]
        out["energies"] = energies
    return out


def _phase_fractions(st0, st1):
    tot = np.zeros(len(PHASES))
    for a, b in zip(st0, st1):
        tot += np.asarray(b["phase_ticks"][:len(PHASES)], dtype=np.float64) - np.asarray(
            a["phase_ticks"][:len(PHASES)], dtype=np.float64)
    s = tot.sum()
    return {k: round(float(v / s), 4) if s > 0 else 0.0 for k, v in zip(PHASES, tot)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--sizes", default="686", help="comma-separated n = 2K^3")
    ap.add_argument("--walkers", type=int, default=64)
    ap.add_argument("--sweeps", type=int, default=120)
    ap.add_argument("--discard", type=int, default=20)
    ap.add_argument("--step", type=float, default=0.55)
    ap.add_argument("--permtol", type=float, default=0.05)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--chunks", type=int, default=1,
                    help="launches per sweep (progress lines in between, for large n)")
    a = ap.parse_args(argv)
    for n in [int(x) for x in a.sizes.split(",")]:
        K = round((n / 2) ** (1.0 / 3.0))
        if 2 * K ** 3 != n:
            raise SystemExit(f"n = {n} is not 2K^3")
        r = run(K, a.walkers, a.sweeps, a.discard, step=a.step, permtol=a.permtol,
                autotune=not a.no_autotune, chunks=a.chunks,
                progress=lambda s: print(f"sweep {s + 1}/{a.sweeps}", file=sys.stderr, flush=True),
                note=lambda text: print(text, file=sys.stderr, flush=True))
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
