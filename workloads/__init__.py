"""Seeded, synthetic inputs shared by the oracle and the GPU path.

This module holds *inputs only*: lattice bond lists of the spin models the
paper studies, the run parameters of each workload, and seeded Gaussian draws.
It contains none of the method's arithmetic (no MPO construction, no
contraction, no eigen- or singular-value step); both the oracle and the GPU
driver build everything else from these inputs with their own code.

Conventions used by every consumer:

* Sites are numbered 1, 2, 3, ... along the one-dimensional path of the matrix
  product state; the Hamiltonian is periodic with an l-site unit cell (l even).
* A model is given by ``cell_bonds``: a list of ``(k, k2, J)`` with
  ``1 <= k <= l`` and ``k2 > k``, meaning the term ``J * s_k . s_k2``; the full
  infinite Hamiltonian is the sum of these terms translated by every multiple
  of l (the periodic l-site MPO of the paper's Sec. 3, Eq. (7)).
* Charges are 2*S^z.  The local basis of a spin-1/2 is ``[up, down]`` with
  charges ``[+1, -1]``.
"""
from __future__ import annotations

import json
import math

import numpy as np

SEED = 1606

# --------------------------------------------------------------------------
# Lattices (the paper's benchmark model is the Heisenberg model sum s_i.s_j,
# Sec. 4; the chain, random chain and square cylinder are the smaller
# workloads of the same family).
# --------------------------------------------------------------------------


def chain_bonds(ell: int, J=1.0):
    """Nearest-neighbour chain: J_k couples sites k and k+1 (k = 1..l).

    ``J`` is a scalar or a length-l sequence (bond k uses J[k-1]).  Bonds with
    J == 0 are omitted, so the dimerised limit has fewer MPO channels.
    """
    Js = np.broadcast_to(np.asarray(J, dtype=np.float64), (ell,))
    return [(k, k + 1, float(Js[k - 1])) for k in range(1, ell + 1) if Js[k - 1] != 0.0]


def dimerised_bonds(ell: int):
    """J_odd = 1, J_even = 0: isolated singlet pairs (2j-1, 2j)."""
    return chain_bonds(ell, [1.0 if k % 2 == 1 else 0.0 for k in range(1, ell + 1)])


def random_chain_couplings(ell: int = 16, lo: float = 0.5, hi: float = 1.5):
    """Seeded i.i.d. uniform couplings J_1..J_l of the random-bond chain."""
    return np.random.default_rng([SEED, 3]).uniform(lo, hi, ell)


def random_chain_bonds(ell: int = 16):
    return chain_bonds(ell, random_chain_couplings(ell))


def yc4_square_bonds(J: float = 1.0):
    """Square-lattice cylinder of circumference 4, snake path, l = 8 (two columns).

    Site (x, y), y in 0..3 periodic, has path index 4x + k + 1 where k runs
    over y ascending for even x and descending for odd x.  Bonds:
    (x,y)-(x,y+1 mod 4) and (x,y)-(x+1,y).
    """
    def idx(x, y):
        k = y if x % 2 == 0 else 3 - y
        return 4 * x + k + 1

    bonds = {}
    for x in range(2):
        for y in range(4):
            for (x2, y2) in ((x, (y + 1) % 4), (x + 1, y)):
                a, b = idx(x, y), idx(x2, y2)
                k, k2 = min(a, b), max(a, b)
                if k > 8:
                    continue
                bonds[(k, k2)] = bonds.get((k, k2), 0.0) + J
    return sorted((k, k2, J_) for (k, k2), J_ in bonds.items())


def yc8_kagome_bonds(J: float = 1.0):
    """Kagome cylinder YC8 on a 12-site unit cell (one ring of 12 sites).

    Ring r holds sites 12r+1..12r+12.  For c = 0..3 the bond classes are
    (3c+1,3c+2), (3c+2,3c+3), (3c+3,3c+4), (3c+2,3c+4) inside the ring, with
    index 13 wrapping to 1 inside the ring, and (3c+3,3c+13), (3c+3,3c+14)
    to the next ring.  These are the six classes whose bond strengths the
    paper lists in Sec. 4 (bond strength subsection), repeated around the
    circumference with period 3.
    """
    bonds = {}

    def add(a, b):
        k, k2 = min(a, b), max(a, b)
        bonds[(k, k2)] = bonds.get((k, k2), 0.0) + J

    def ring(a):  # wrap inside ring 0
        return (a - 1) % 12 + 1

    for c in range(4):
        add(3 * c + 1, 3 * c + 2)
        add(3 * c + 2, 3 * c + 3)
        add(3 * c + 3, ring(3 * c + 4))
        add(3 * c + 2, ring(3 * c + 4))
        add(3 * c + 3, 3 * c + 13)
        add(3 * c + 3, 3 * c + 14)
    return sorted((k, k2, J_) for (k, k2), J_ in bonds.items())


def yc8_bond_classes():
    """The six nearest-neighbour bond classes of the YC8 cylinder whose strengths Sec. 4 reports, each as its four
    translates by 3 sites around the circumference (site labels; inside a ring the index wraps, a label above 12
    is a site of the next ring).  Class names are those of the paper: (1,2), (2,3), (3,4), (2,4), (3,13), (3,14)."""
    def ring(a):
        return (a - 1) % 12 + 1
    rules = {"1-2": lambda c: (3 * c + 1, 3 * c + 2), "2-3": lambda c: (3 * c + 2, 3 * c + 3),
             "3-4": lambda c: (3 * c + 3, ring(3 * c + 4)), "2-4": lambda c: (3 * c + 2, ring(3 * c + 4)),
             "3-13": lambda c: (3 * c + 3, 3 * c + 13), "3-14": lambda c: (3 * c + 3, 3 * c + 14)}
    return {name: [tuple(sorted(f(c))) for c in range(4)] for name, f in rules.items()}


def yc8_axis_sweep(rings: int, label: int = 2):
    """Sites on the straight line along the YC8 cylinder's axis through site `label` of ring 0, one per ring
    R = 0..rings, with their distance from it (nearest-neighbour distance 1).

    Embedding (reconstructed; the paper shows it only in its figure): kagome Bravais vectors of length 2 at 60
    degrees, a1 wrapped four times around the circumference, a2 from one ring to the next, so a2 moves sqrt(3)
    along the axis and one unit (half of a1) around.  Site 3c + s + 1 (s = 0, 1, 2) of a ring is sublattice s of
    the c-th kagome cell around it.  The point of ring R on the line is R a2 - floor(R / 2) a1: cell c - floor(R/2)
    (mod 4), at distance sqrt(3 R^2 + (R mod 2)^2).  For label 2 this gives the sweep 2, 14, 35, 47, ... of the
    correlation-length subsection of Sec. 4."""
    c0, sub = divmod(label - 1, 3)
    out = []
    for R in range(rings + 1):
        c = (c0 - R // 2) % 4
        out.append((12 * R + 3 * c + sub + 1, math.sqrt(3 * R * R + (R % 2))))
    return out


def segment_bonds(cell_bonds, ell: int, first: int, last: int):
    """All bonds (i, j, J) of the infinite periodic model with first <= i < j <= last."""
    out = {}
    tmin = (first - ell - 1) // ell - 1
    tmax = last // ell + 1
    for (k, k2, J) in cell_bonds:
        for t in range(tmin, tmax + 1):
            i, j = k + t * ell, k2 + t * ell
            if first <= i and j <= last:
                out[(i, j)] = out.get((i, j), 0.0) + J
    return sorted((i, j, J) for (i, j), J in out.items())


# --------------------------------------------------------------------------
# Workloads.  Parameters follow the five benchmark configurations: a uniform
# chain (l=4, m=32), a matvec microbenchmark, a random-bond chain (l=16,
# m=256), a YC4 square cylinder (l=8, m=1024) and a YC8 kagome cylinder
# (l=12, m=2048/4096).
# --------------------------------------------------------------------------

# lam_floor: Schmidt values at or below it count as zero (selection and the lambda = 0 branch of
# Eq. (10)).  It lies above the numerical noise of a computed two-site state (Lanczos residual
# 1e-8; measured noise tails of the spectra reach 1e-9), so that whether a value is zero does not
# depend on rounding.
COMMON = dict(tol_E=1e-12, tol_res=1e-8, k_max=300, lam_floor=1e-8, deg_rel=1e-5, u1=True)


def workload(name: str, **over):
    """Run parameters of a named workload (a plain dict)."""
    if name == "chain":
        cfg = dict(name="chain", ell=4, bonds=chain_bonds(4), m=32, n_max=20, prec="f64")
    elif name == "random_chain":
        cfg = dict(name="random_chain", ell=16, bonds=random_chain_bonds(16), m=256, n_max=64,
                   prec="f64")
    elif name == "yc4":
        cfg = dict(name="yc4", ell=8, bonds=yc4_square_bonds(), m=1024, n_max=40, prec="f32")
    elif name == "yc8":
        cfg = dict(name="yc8", ell=12, bonds=yc8_kagome_bonds(), m=2048, n_max=36, prec="bf16x3")
    elif name == "dimer":
        cfg = dict(name="dimer", ell=4, bonds=dimerised_bonds(4), m=8, n_max=8, prec="f64")
    else:
        raise KeyError(name)
    out = dict(COMMON)
    out.update(cfg)
    out.update(over)
    return out


# Keys of a run configuration, with their types.  `seed` (optional) seeds the random start vectors of the first
# two iterations; without it they come from SEED.
CONFIG_KEYS = dict(name=str, ell=int, bonds=list, m=int, n_max=int, prec=str, tol_E=float, tol_res=float, k_max=int,
                   lam_floor=float, deg_rel=float, u1=bool, seed=int)
PRECISIONS = ("f64", "f32", "bf16x3")


def check_config(cfg: dict) -> dict:
    """The configuration with its bonds as (k, k2, J) tuples, after checking its keys, types and values; raises
    ValueError on anything else."""
    missing = [k for k in CONFIG_KEYS if k != "seed" and k not in cfg]
    unknown = [k for k in cfg if k not in CONFIG_KEYS]
    if missing or unknown:
        raise ValueError(f"configuration: missing {missing}, unknown {unknown}")
    out = {}
    for k, v in cfg.items():
        t = CONFIG_KEYS[k]
        if t is float and isinstance(v, int) and not isinstance(v, bool):
            v = float(v)
        if not isinstance(v, t) or (t is int and isinstance(v, bool)):
            raise ValueError(f"configuration: {k} must be {t.__name__}, not {type(v).__name__}")
        out[k] = v
    ell = out["ell"]
    if ell < 2 or ell % 2:
        raise ValueError("configuration: ell must be even and at least 2")
    bonds = []
    for b in out["bonds"]:
        if len(b) != 3:
            raise ValueError(f"configuration: bond {b} is not (k, k2, J)")
        k, k2, J = int(b[0]), int(b[1]), float(b[2])
        if k != b[0] or k2 != b[1] or not 1 <= k <= ell or k2 <= k:
            raise ValueError(f"configuration: bond {b} needs integer sites with 1 <= k <= ell and k2 > k")
        bonds.append((k, k2, J))
    if not bonds:
        raise ValueError("configuration: no bonds")
    out["bonds"] = bonds
    if out["prec"] not in PRECISIONS:
        raise ValueError(f"configuration: prec must be one of {PRECISIONS}")
    if out["m"] < 1 or out["n_max"] < 1 or out["k_max"] < 1:
        raise ValueError("configuration: m, n_max and k_max must be positive")
    return out


def save_config(cfg: dict, path: str) -> None:
    """Write a run configuration as one JSON object (bonds as [k, k2, J] lists)."""
    c = check_config(dict(cfg))
    with open(path, "w") as f:
        json.dump(dict(c, bonds=[list(b) for b in c["bonds"]]), f, indent=1)
        f.write("\n")


def load_config(path: str) -> dict:
    """A run configuration from a JSON file written by save_config (or by hand, with the same keys)."""
    with open(path) as f:
        return check_config(json.load(f))


# --------------------------------------------------------------------------
# Seeded random numbers.  Random numbers the method draws (the start vector
# of the first two iterations) are produced here and passed to both sides.
# --------------------------------------------------------------------------


def start_vector(n_elem: int, n: int, i: int, seed: int = SEED):
    """Gaussian N(0,1) start vector for superblock i at iteration n (n = 1, 2).

    ``n_elem`` is the number of stored elements of the two-site state in its
    canonical block order; the caller fills the blocks in that order.
    """
    return np.random.default_rng([seed, n, i]).standard_normal(n_elem)


def gaussian(n_elem: int, *key):
    """Generic seeded N(0,1) draw keyed by ``(SEED, *key)``."""
    return np.random.default_rng([SEED, *key]).standard_normal(n_elem)


def sector_dims(m: int, qmax: int = 10, width: float = 8.0):
    """Bond sectors of the matvec microbenchmark.

    Charges q in {-qmax, ..., qmax} step 2 with dims proportional to
    exp(-(q/2)^2 / width), rounded by largest remainder to sum to m.
    Returns (charges, dims) with zero-dim sectors removed.
    """
    qs = np.arange(-qmax, qmax + 1, 2)
    w = np.exp(-((qs / 2.0) ** 2) / width)
    raw = m * w / w.sum()
    base = np.floor(raw).astype(int)
    rem = m - base.sum()
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    keep = base > 0
    return [int(q) for q in qs[keep]], [int(d) for d in base[keep]]


def bethe_ansatz_energy():
    """Ground-state energy per site of the infinite uniform spin-1/2 chain, 1/4 - ln 2."""
    return 0.25 - math.log(2.0)
