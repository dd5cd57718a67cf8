"""Seeded synthetic workloads: reaction networks, initial states, horizons,
snapshot grids and parameter-set tables.

This module only *describes inputs*. It holds none of the simulation
arithmetic, imports neither the GPU binding nor the oracle, and is the one
place both sides take their inputs from.

Networks (Kimpson, Flegg & Flegg, Sec. 4):
  birth-death (Sec. 4.1), Schloegl (Sec. 4.2), telegraph (Sec. 4.3),
  dimerisation (Sec. 4.4; the closed 2A <-> D form, plus the open form with
  birth and death of the monomer), repressilator (Sec. 4.5, Hill-regulated
  transcription f(P) = a0 + a / (1 + (P/K)^h)).

Mass-action convention: a reaction with reactant orders o_s has propensity
a = k * prod_s binom(x_s, o_s) = (k / prod_s o_s!) * prod_s x_s (x_s - 1) ... (x_s - o_s + 1).
Reservoir species (Schloegl's A and B) are folded into k by the caller, as in
the paper's rescaling argument (Sec. 4.2: only k1*A and k3*B matter).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

LAW_MASS_ACTION = 0
LAW_HILL_REPRESS = 1
LAW_HILL_ACTIVATE = 2


@dataclass(frozen=True)
class ModelSpec:
    """A reaction network: M reactions over N species."""
    name: str
    species: tuple
    order: np.ndarray      # [M, N] int32 reactant orders (mass action)
    nu: np.ndarray         # [M, N] int32 net change
    law: np.ndarray        # [M] int32
    rate: np.ndarray       # [M] float64: mass action k_j, Hill v_j
    hill_reg: np.ndarray   # [M] int32 regulator species (Hill)
    hill_h: np.ndarray     # [M] int32 Hill exponent
    hill_b: np.ndarray     # [M] float64 basal rate (Hill)
    hill_K: np.ndarray     # [M] float64 half-saturation constant (Hill)

    @property
    def n_species(self) -> int:
        return len(self.species)

    @property
    def n_reactions(self) -> int:
        return int(self.law.shape[0])


def _build(name, species, reactions):
    """reactions: list of dicts with keys 'reactants' {sp: order}, 'change'
    {sp: delta} and either 'k' (mass action) or 'hill' (kind, reg, b, v, K, h)."""
    N, M = len(species), len(reactions)
    ix = {s: i for i, s in enumerate(species)}
    order = np.zeros((M, N), np.int32)
    nu = np.zeros((M, N), np.int32)
    law = np.zeros(M, np.int32)
    rate = np.zeros(M, np.float64)
    reg = np.zeros(M, np.int32)
    hh = np.ones(M, np.int32)
    hb = np.zeros(M, np.float64)
    hK = np.ones(M, np.float64)
    for j, r in enumerate(reactions):
        for s, o in r.get("reactants", {}).items():
            order[j, ix[s]] = o
        for s, d in r.get("change", {}).items():
            nu[j, ix[s]] = d
        if "hill" in r:
            kind, rg, b, v, K, h = r["hill"]
            law[j] = LAW_HILL_REPRESS if kind == "repress" else LAW_HILL_ACTIVATE
            reg[j], hb[j], rate[j], hK[j], hh[j] = ix[rg], b, v, K, h
        else:
            law[j] = LAW_MASS_ACTION
            rate[j] = r["k"]
    return ModelSpec(name, tuple(species), order, nu, law, rate, reg, hh, hb, hK)


def birth_death(kb: float = 10.0, kd: float = 0.1) -> ModelSpec:
    """0 -> X at kb; X -> 0 at kd*X."""
    return _build("birth_death", ["X"], [
        {"change": {"X": +1}, "k": kb},
        {"reactants": {"X": 1}, "change": {"X": -1}, "k": kd},
    ])


def schlogl(c1=3e-7, c2=1e-4, c3=1e-3, c4=3.5, A=1e5, B=2e5) -> ModelSpec:
    """a1 = c1 A X(X-1)/2, a2 = c2 X(X-1)(X-2)/6, a3 = c3 B, a4 = c4 X;
    stoichiometry +1, -1, +1, -1."""
    return _build("schlogl", ["X"], [
        {"reactants": {"X": 2}, "change": {"X": +1}, "k": c1 * A},
        {"reactants": {"X": 3}, "change": {"X": -1}, "k": c2},
        {"change": {"X": +1}, "k": c3 * B},
        {"reactants": {"X": 1}, "change": {"X": -1}, "k": c4},
    ])


def telegraph(k_on=0.05, k_off=0.1, k_m=20.0, beta=1.0) -> ModelSpec:
    """G_off -> G_on (k_on), G_on -> G_off (k_off), G_on -> G_on + M (k_m),
    M -> 0 (beta*M)."""
    return _build("telegraph", ["G_off", "G_on", "M"], [
        {"reactants": {"G_off": 1}, "change": {"G_off": -1, "G_on": +1}, "k": k_on},
        {"reactants": {"G_on": 1}, "change": {"G_on": -1, "G_off": +1}, "k": k_off},
        {"reactants": {"G_on": 1}, "change": {"M": +1}, "k": k_m},
        {"reactants": {"M": 1}, "change": {"M": -1}, "k": beta},
    ])


def dimer_open(k1=50.0, k2=0.1, k3=0.001, k4=0.5) -> ModelSpec:
    """0 -> M (k1), M -> 0 (k2 M), 2M -> D (k3 M(M-1)/2), D -> 2M (k4 D)."""
    return _build("dimer_open", ["M", "D"], [
        {"change": {"M": +1}, "k": k1},
        {"reactants": {"M": 1}, "change": {"M": -1}, "k": k2},
        {"reactants": {"M": 2}, "change": {"M": -2, "D": +1}, "k": k3},
        {"reactants": {"D": 1}, "change": {"M": +2, "D": -1}, "k": k4},
    ])


def dimer_closed(kf=1e-3, kr=0.1) -> ModelSpec:
    """2A -> D at kf A(A-1)/2, D -> 2A at kr D (Sec. 4.4)."""
    return _build("dimer_closed", ["A", "D"], [
        {"reactants": {"A": 2}, "change": {"A": -2, "D": +1}, "k": kf},
        {"reactants": {"D": 1}, "change": {"A": +2, "D": -1}, "k": kr},
    ])


def repressilator(alpha0=0.05, alpha=50.0, K=40.0, h=2, dm=1.0, beta=5.0, dp=0.2) -> ModelSpec:
    """Three genes; m_i made at alpha0 + alpha/(1 + (p_{i-1}/K)^h), decays at dm;
    p_i made at beta*m_i, decays at dp. Species order (m0, m1, m2, p0, p1, p2);
    reactions gene by gene: transcription, mRNA decay, translation, protein decay."""
    sp = ["m0", "m1", "m2", "p0", "p1", "p2"]
    rx = []
    for i in range(3):
        m, p, rep = f"m{i}", f"p{i}", f"p{(i - 1) % 3}"
        rx += [
            {"change": {m: +1}, "hill": ("repress", rep, alpha0, alpha, K, h)},
            {"reactants": {m: 1}, "change": {m: -1}, "k": dm},
            {"reactants": {m: 1}, "change": {p: +1}, "k": beta},
            {"reactants": {p: 1}, "change": {p: -1}, "k": dp},
        ]
    return _build("repressilator", sp, rx)


def self_repressor(b=2.0, v=30.0, K=10.0, h=2, d=1.0) -> ModelSpec:
    """0 -> X at b + v/(1 + (X/K)^h); X -> 0 at d X. A one-species chain whose
    stationary law follows from detailed balance (used to pin the Hill law)."""
    return _build("self_repressor", ["X"], [
        {"change": {"X": +1}, "hill": ("repress", "X", b, v, K, h)},
        {"reactants": {"X": 1}, "change": {"X": -1}, "k": d},
    ])


def snapshot_grid(t_end: float, n_snap: int) -> np.ndarray:
    """n_snap evenly spaced times 0 .. t_end: t_k = (k * t_end) / (n_snap - 1);
    the last one equals t_end exactly."""
    if n_snap == 1:
        return np.array([float(t_end)])
    k = np.arange(n_snap, dtype=np.float64)
    return (k * float(t_end)) / float(n_snap - 1)


def dimer_sweep_rates(n_sets: int = 4096, seed: int = 7, base=(50.0, 0.1, 0.001, 0.5)) -> np.ndarray:
    """[n_sets, 4] rates, each base value times 10^(2u - 1), u ~ U(0,1) from
    numpy's PCG64 generator seeded with ``seed``: log-uniform over +-1 decade."""
    rng = np.random.default_rng(seed)
    u = rng.random((n_sets, len(base)))
    return np.asarray(base, dtype=np.float64)[None, :] * np.power(10.0, 2.0 * u - 1.0)


@dataclass
class Item:
    """One model's share of an ensemble run."""
    model: ModelSpec
    x0: np.ndarray
    n_traj: int
    set_rate: np.ndarray | None = None   # [n_sets, M] or None
    traj_per_set: int = 0


@dataclass
class Workload:
    name: str
    items: list
    t_end: float
    snap_t: np.ndarray
    seed: int
    modes: tuple
    max_events: int
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_traj(self) -> int:
        return sum(it.n_traj for it in self.items)


def config_birth_death(n_traj: int = 10_000) -> Workload:
    """Birth-death, kb=10, kd=0.1, X0=0, T_end=100, one snapshot at 100,
    10,000 trajectories, seed 1; stationary law Poisson(100)."""
    return Workload("birth_death", [Item(birth_death(), np.array([0], np.int32), n_traj)],
                    100.0, np.array([100.0]), 1, ("FP64",), 1900 * 64)


def config_schlogl(n_traj: int = 100_000) -> Workload:
    """Schloegl bistable: X0=250, T_end=10, 101 evenly spaced snapshots,
    100,000 trajectories; FP64 vs mixed FP16 (RTN and SR)."""
    return Workload("schlogl", [Item(schlogl(), np.array([250], np.int32), n_traj)],
                    10.0, snapshot_grid(10.0, 101), 1,
                    ("FP64", "MIX_F16_SR", "MIX_F16_RTN", "MIX_BF16_SR"), 43_574 * 64)


def config_telegraph(n_traj: int = 1_000_000) -> Workload:
    """Telegraph: gene off, M=0, T_end=200, snapshots every 1.0,
    1,000,000 trajectories; uniform FP16/BF16 x {RTN, SR, SR+norm}."""
    return Workload("telegraph", [Item(telegraph(), np.array([1, 0, 0], np.int32), n_traj)],
                    200.0, snapshot_grid(200.0, 201), 1,
                    ("FP64", "UNI_F16_RTN", "UNI_F16_SR", "UNI_F16_SR_NORM",
                     "UNI_BF16_RTN", "UNI_BF16_SR", "UNI_BF16_SR_NORM"), 2584 * 64)


def config_dimer_sweep(n_sets: int = 4096, traj_per_set: int = 256) -> Workload:
    """Open dimerisation, 4,096 log-uniform parameter sets (seed 7) x 256
    trajectories, M0=D0=0, T_end=50, snapshots every 1.0; one persistent launch."""
    rates = dimer_sweep_rates(n_sets)
    it = Item(dimer_open(), np.array([0, 0], np.int32), n_sets * traj_per_set, rates, traj_per_set)
    return Workload("dimer_sweep", [it], 50.0, snapshot_grid(50.0, 51), 1,
                    ("FP64", "MIX_F16_SR"), 3_000_000)


def config_heterogeneous(n_traj_total: int = 4_000_000) -> Workload:
    """All five networks in one launch, split evenly, T_end=500, snapshots
    every 1.0: birth-death (X0=0), Schloegl (X0=250), telegraph (gene off),
    open dimer at base rates (M0=D0=0), repressilator (m=0, p=(0,0,20))."""
    per = n_traj_total // 5
    items = [
        Item(birth_death(), np.array([0], np.int32), per),
        Item(schlogl(), np.array([250], np.int32), per),
        Item(telegraph(), np.array([1, 0, 0], np.int32), per),
        Item(dimer_open(), np.array([0, 0], np.int32), per),
        Item(repressilator(), np.array([0, 0, 0, 0, 0, 20], np.int32), per),
    ]
    return Workload("heterogeneous", items, 500.0, snapshot_grid(500.0, 501), 1,
                    ("FP64", "MIX_BF16_SR", "MIX_F16_SR"), 250_000_000)


CONFIGS = {
    "birth_death": config_birth_death,
    "schlogl": config_schlogl,
    "telegraph": config_telegraph,
    "dimer_sweep": config_dimer_sweep,
    "heterogeneous": config_heterogeneous,
}
