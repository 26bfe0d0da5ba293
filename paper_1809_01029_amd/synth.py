"""Seeded synthetic inputs: chemical mechanisms and thermochemical state batches.

This module only *constructs inputs*.  It holds none of the arithmetic that the
source-term / Jacobian path computes (no rate constants, no equilibrium
constants, no rates of progress, no derivatives).  Both the GPU library and the
CPU oracle read what it writes, and nothing else is shared between them.

What it builds (all from ``numpy.random.Generator(PCG64(seed))``):

* Species: C/H/O/N atom counts drawn in 0..4 with 1..6 atoms in total
  (rejection), isomers allowed.  The last species is the bath gas (N2-like),
  which the paper's state vector excludes (Sec. 2.2, state vector) and which
  takes part in few reactions, as a bath gas usually does.
* Thermodynamics: two-range NASA 7-coefficient polynomials fitted by least
  squares to a smooth random Cp(T)/R on [300, 1000] K and [1000, 5000] K, the
  high range constrained to the low one at 1000 K so that Cp, H and S are
  continuous there.  Formation enthalpy H(298.15)/R ~ U[-3e4, 3e4] K and
  S(298.15)/R ~ U[20, 40].
* Reactions: element-balanced by construction (a product multiset is drawn
  among the multisets with the same element-count vector as the reactants),
  molecularity <= 3 per side, stoichiometric coefficients 1 or 2.  Species
  popularity follows a Zipf-like law so that the Jacobian sparsity falls near
  the exact-Jacobian densities the paper reports for models of the same size
  (Sec. 3.4, Table of Jacobian densities).  Type mix per workload: reversible
  elementary, irreversible elementary, third-body (efficiencies U[0.5, 5] on
  1..6 species), Lindemann and Troe falloff (alpha U[0,1], T***, T*, T** in
  U[100, 5000] K).  Arrhenius: log10 A ~ U[8,16], b ~ U[-2,3], Ea/R ~
  U[0, 30000] K; falloff low-pressure limits drawn from the same ranges.
  Optional further types (absent from the default mixes): SRI falloff
  (a U[0.1, 2], b and c U[100, 2000] K, d U[0.5, 2], e U[-0.5, 0.5]);
  chemically activated reactions (Lindemann, Troe or SRI form); pressure-
  dependent Arrhenius (P-Log: 2..5 pressures with log10 P/atm in [-1, 2.5],
  each with the reaction's Arrhenius perturbed by U[-2, 2] in ln A,
  U[-0.5, 0.5] in b and U[-2000, 2000] K in Ea/R); Chebyshev (3..6 x 2..4
  coefficients over 290..3000 K and 0.01..100 atm, alpha_00 U[8, 13],
  alpha_10 U[-3, 0], the others N(0, 0.3^2)/(1 + t + p)).
* States: T ~ U[Tlo, Thi], P ~ U[Plo, Phi] atm, mass fractions
  Y ~ Dirichlet(0.5), V = 1 m^3, moles from the ideal-gas law.  The same draw
  gives the constant-pressure state (T, V, n_1..n_{Ns-1}) with parameter P and
  the constant-volume state (T, P, n_1..n_{Ns-1}) with parameter V.

The mechanism description format (text, one record per line, every real
written with 17 significant digits so it round-trips exactly)::

    PJMECH 1
    SPECIES <Ns>
    SP <k> <name> <W> <nC> <nH> <nO> <nN> <Tlow> <Tmid> <Thigh> <a_lo x7> <a_hi x7>
    REACTIONS <Nr>
    RX <i> <TYPE> <rev> <n_reac> (<sp> <nu>)* <n_prod> (<sp> <nu>)* <lnA> <b> <Ea/R>
       [LOW <lnA0> <b0> <Ea0/R>] [TROE <alpha> <T***> <T*> <T**>] [SRI <a> <b> <c> <d> <e>]
       [CHEMACT] [PLOG <m> (<P> <lnA> <b> <Ea/R>)*]
       [CHEB <NT> <NP> <Tmin> <Tmax> <Pmin> <Pmax> <alpha_tp, t-major>] [EFF <m> (<sp> <alpha>)*]
    END

TYPE is ELEM, THREEBODY, LINDEMANN, TROE, SRI, PLOG or CHEB; rev is 1
(reversible) or 0.  Species indices are 0-based; the last species is the bath
gas.  For LINDEMANN, TROE and SRI the main Arrhenius is the high-pressure
limit and LOW the low-pressure one; CHEMACT marks a chemically activated
reaction (the rate multiplies the low-pressure limit).  For PLOG and CHEB the
main Arrhenius is a factor on the tabulated rate constant (0 0 0 = none);
pressures are in Pa, in ascending order for PLOG.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

ATOMIC_WEIGHTS = (12.011, 1.008, 15.999, 14.007)  # C, H, O, N  [kg/kmol]
ELEMENTS = ("C", "H", "O", "N")
ATM = 101325.0  # Pa
R_GAS = 8314.462618  # J/(kmol K); used here only to turn mole fractions into moles

T_LOW, T_MID, T_HIGH = 300.0, 1000.0, 5000.0

TYPES = ("ELEM", "THREEBODY", "LINDEMANN", "TROE", "SRI", "PLOG", "CHEB")
FALLOFF_TYPES = ("LINDEMANN", "TROE", "SRI")


@dataclasses.dataclass
class Reaction:
    type: str                      # one of TYPES
    rev: bool
    reac: List[Tuple[int, int]]    # (species, nu')
    prod: List[Tuple[int, int]]    # (species, nu'')
    lnA: float
    b: float
    theta: float                   # Ea / R  [K]
    low: Optional[Tuple[float, float, float]] = None      # (lnA0, b0, theta0)
    troe: Optional[Tuple[float, float, float, float]] = None  # (alpha, T***, T*, T**)
    eff: List[Tuple[int, float]] = dataclasses.field(default_factory=list)
    sri: Optional[Tuple[float, float, float, float, float]] = None  # (a, b, c, d, e)
    chemact: bool = False          # chemically activated (falloff forms)
    plog: Optional[List[Tuple[float, float, float, float]]] = None  # (P [Pa], lnA, b, Ea/R)
    # Chebyshev: ((Tmin, Tmax, Pmin [Pa], Pmax [Pa]), coefficients [NT][NP])
    cheb: Optional[Tuple[Tuple[float, float, float, float], List[List[float]]]] = None


@dataclasses.dataclass
class Mechanism:
    names: List[str]
    W: np.ndarray            # (Ns,) molecular weights
    comp: np.ndarray         # (Ns, 4) int atom counts C,H,O,N
    tmid: np.ndarray         # (Ns,)
    a_lo: np.ndarray         # (Ns, 7)
    a_hi: np.ndarray         # (Ns, 7)
    reactions: List[Reaction]

    @property
    def n_species(self) -> int:
        return len(self.names)

    @property
    def n_reactions(self) -> int:
        return len(self.reactions)

    @property
    def state_size(self) -> int:
        return self.n_species + 1


# ----------------------------------------------------------------------------
# workloads

@dataclasses.dataclass(frozen=True)
class MixSpec:
    third_body: float = 0.10
    falloff: float = 0.15          # half Lindemann, half Troe
    irreversible: float = 0.05
    sri: float = 0.0               # SRI falloff
    chem_act: float = 0.0          # chemically activated (Lindemann, Troe, SRI in turn)
    plog: float = 0.0
    cheb: float = 0.0


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    ns: int
    nr: int
    n_states: int
    mech_seed: int
    state_seed: int
    T_range: Tuple[float, float] = (600.0, 2200.0)
    P_range_atm: Tuple[float, float] = (1.0, 50.0)
    mix: MixSpec = MixSpec()
    zipf: float = 1.0
    bath_reactions: int = 0
    n_inert: int = 0


# Sizes of the four models the paper benchmarks (H2/CO, GRI-Mech 3.0,
# USC-Mech II, iC5H11OH) stand in as synthetic mechanisms of the same size.
WORKLOADS: Dict[str, Workload] = {
    "ns13": Workload("ns13", 13, 27, 1024, 13, 1013, zipf=1.5, bath_reactions=1, n_inert=2),
    "ns53": Workload("ns53", 53, 325, 1_048_576, 53, 1053, zipf=2.2, bath_reactions=1, n_inert=1),
    "ns111": Workload("ns111", 111, 784, 262_144, 111, 1111, zipf=2.5, bath_reactions=1, n_inert=2),
    "ns360": Workload("ns360", 360, 2170, 16_384, 360, 1360, T_range=(700.0, 1800.0),
                      P_range_atm=(10.0, 60.0), mix=MixSpec(0.10, 0.20, 0.05),
                      zipf=1.2, bath_reactions=2, n_inert=2),
    # the 111-species size with every reaction type the library supports
    "ns111x": Workload("ns111x", 111, 784, 262_144, 111, 1111, zipf=2.5, bath_reactions=1,
                       n_inert=2, mix=MixSpec(third_body=0.10, falloff=0.10, irreversible=0.05,
                                              sri=0.03, chem_act=0.04, plog=0.05, cheb=0.03)),
}


# ----------------------------------------------------------------------------
# species

def _valid_comp(c: np.ndarray) -> bool:
    return bool(np.all(c >= 0) and np.all(c <= 4) and 1 <= int(c.sum()) <= 6)


def _draw_compositions(rng: np.random.Generator, n: int, p_uniform: float = 0.25) -> np.ndarray:
    """Atom counts in 0..4 per element and 1..6 atoms per species.

    Independent uniform draws almost never admit element-balanced reactions
    among a dozen species, so the first species are small fragments (one or
    two atoms, every element represented) and each later species is, with
    probability 1 - p_uniform, the sum or the difference of two species
    already drawn (kept only if it still satisfies the count limits), as
    fragments and their combinations do in real mechanisms.  Repeated
    compositions (isomers) are kept with probability 0.3 per draw.
    """
    out = np.zeros((n, 4), dtype=np.int64)
    if n >= 12:
        n_seed = 5
        for k in range(n_seed):
            c = np.zeros(4, dtype=np.int64)
            c[k % 4] = 1
            if rng.uniform() < 0.5:
                c[rng.integers(0, 4)] += 1
            out[k] = c
    else:
        # few species: fewer, single-atom fragments of randomly chosen elements
        n_seed = max(2, n // 3)
        elems = rng.permutation(4)
        for k in range(n_seed):
            out[k, elems[k % 4]] = 1
    k = n_seed
    while k < n:
        c = None
        if rng.uniform() >= p_uniform:
            for _ in range(64):
                a, b = rng.integers(0, k, size=2)
                cand = out[a] + out[b] if rng.uniform() < 0.6 else out[a] - out[b]
                if _valid_comp(cand):
                    c = cand
                    break
        if c is None:
            while True:
                cand = rng.integers(0, 5, size=4)
                if _valid_comp(cand):
                    c = cand
                    break
        if np.any(np.all(out[:k] == c[None, :], axis=1)) and rng.uniform() >= 0.3:
            continue
        out[k] = c
        k += 1
    return out


def _cp_target(rng: np.random.Generator, atoms: int):
    """A smooth random Cp(T)/R: constant 2.5 for one atom, otherwise rising
    monotonically from about 3.5 towards about 3*atoms - 2."""
    if atoms == 1:
        return lambda T: np.full_like(np.asarray(T, dtype=float), 2.5)
    c0 = 3.5 + rng.uniform(-0.3, 0.5)
    c1 = max(c0 + 0.5, 3.0 * atoms - 2.0 + rng.uniform(-0.5, 0.5))
    tc = rng.uniform(600.0, 1800.0)
    w = rng.uniform(400.0, 1200.0)

    def f(T):
        T = np.asarray(T, dtype=float)
        return c0 + (c1 - c0) * 0.5 * (1.0 + np.tanh((T - tc) / w))

    return f


def _fit_nasa(rng: np.random.Generator, atoms: int, h298: float, s298: float):
    """Least-squares NASA-7 fit of a random Cp/R, continuous at T_MID."""
    f = _cp_target(rng, atoms)
    tl = np.linspace(T_LOW, T_MID, 200)
    th = np.linspace(T_MID, T_HIGH, 400)
    # scaled monomials for conditioning: x = T / 1000
    Al = np.vstack([(tl / 1000.0) ** m for m in range(5)]).T
    cl, *_ = np.linalg.lstsq(Al, f(tl), rcond=None)
    lo = np.array([cl[m] / 1000.0 ** m for m in range(5)])
    cp_mid = sum(lo[m] * T_MID ** m for m in range(5))
    # high range: cp(T) = cp_mid + sum_{m=1..4} d_m ((T/1000)^m - 1)
    Ah = np.vstack([(th / 1000.0) ** m - 1.0 for m in range(1, 5)]).T
    dh, *_ = np.linalg.lstsq(Ah, f(th) - cp_mid, rcond=None)
    hi = np.zeros(5)
    for m in range(1, 5):
        hi[m] = dh[m - 1] / 1000.0 ** m
    hi[0] = cp_mid - sum(hi[m] * T_MID ** m for m in range(1, 5))

    # Integration constants.  H/R = sum a_m T^{m+1}/(m+1) + a6 ;
    # S/R = a_0 ln T + sum_{m>=1} a_m T^m / m + a7.
    def h_int(a, T):
        return sum(a[m] * T ** (m + 1) / (m + 1) for m in range(5))

    def s_int(a, T):
        return a[0] * math.log(T) + sum(a[m] * T ** m / m for m in range(1, 5))

    a6_lo = h298 - h_int(lo, 298.15)
    a7_lo = s298 - s_int(lo, 298.15)
    a6_hi = a6_lo + h_int(lo, T_MID) - h_int(hi, T_MID)
    a7_hi = a7_lo + s_int(lo, T_MID) - s_int(hi, T_MID)
    a_lo = np.concatenate([lo, [a6_lo, a7_lo]])
    a_hi = np.concatenate([hi, [a6_hi, a7_hi]])
    return a_lo, a_hi


# ----------------------------------------------------------------------------
# reactions

_BASE = 32


def _code(c: np.ndarray) -> np.ndarray:
    c = np.asarray(c, dtype=np.int64)
    return ((c[..., 0] * _BASE + c[..., 1]) * _BASE + c[..., 2]) * _BASE + c[..., 3]


class _ProductIndex:
    """Finds every product multiset (size 1..3, coefficients <= 2) whose
    element-count vector equals a given vector.  Candidates come back as an
    (K, 3) index array padded with -1, with their popularity weights."""

    def __init__(self, comp: np.ndarray, allowed: np.ndarray, weight: np.ndarray):
        self.comp = comp
        idx = np.nonzero(allowed)[0]
        self.idx = idx
        self.weight = np.append(weight, 1.0)     # index -1 -> weight 1
        self.code1 = _code(comp[idx])
        ii, jj = np.triu_indices(len(idx))
        self.p_i = idx[ii]
        self.p_j = idx[jj]
        self.pair_comp = comp[self.p_i] + comp[self.p_j]
        self.code2 = _code(self.pair_comp)
        order = np.argsort(self.code1, kind="stable")
        self.sorted_code1 = self.code1[order]
        self.sorted_sp = idx[order]
        self.cache: Dict[int, Tuple[np.ndarray, np.ndarray]] = {}

    def candidates(self, key: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        kc = int(_code(key))
        if kc in self.cache:
            return self.cache[kc]
        rows: List[np.ndarray] = []
        s1 = self.idx[self.code1 == kc]
        rows.append(np.stack([s1, -np.ones_like(s1), -np.ones_like(s1)], axis=1))
        m2 = self.code2 == kc
        rows.append(np.stack([self.p_i[m2], self.p_j[m2], -np.ones(int(m2.sum()), dtype=np.int64)],
                             axis=1))
        need = key[None, :] - self.pair_comp
        ok = np.all(need >= 0, axis=1) & (need.sum(axis=1) >= 1)
        if np.any(ok):
            nc = _code(need[ok])
            pi, pj = self.p_i[ok], self.p_j[ok]
            lo = np.searchsorted(self.sorted_code1, nc, side="left")
            hi = np.searchsorted(self.sorted_code1, nc, side="right")
            cnt = hi - lo
            if cnt.sum():
                rep = np.repeat(np.arange(len(nc)), cnt)
                off = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
                s3 = self.sorted_sp[lo[rep] + off]
                a3, b3 = pi[rep], pj[rep]
                keep = (s3 >= b3) & ~((a3 == b3) & (b3 == s3))   # canonical a<=b<=s, no nu=3
                rows.append(np.stack([a3[keep], b3[keep], s3[keep]], axis=1))
        arr = np.concatenate(rows, axis=0).astype(np.int64)
        w = self.weight[arr].prod(axis=1)
        self.cache[kc] = (arr, w)
        return arr, w


def _multiset(species: Sequence[int]) -> List[Tuple[int, int]]:
    d: Dict[int, int] = {}
    for s in species:
        d[s] = d.get(s, 0) + 1
    return sorted(d.items())


def _draw_arrhenius(rng: np.random.Generator) -> Tuple[float, float, float]:
    log10A = rng.uniform(8.0, 16.0)
    return (log10A * math.log(10.0), rng.uniform(-2.0, 3.0), rng.uniform(0.0, 30000.0))


def make_mechanism(ns: int, nr: int, seed: int, mix: MixSpec = MixSpec(), zipf: float = 1.0,
                   bath_reactions: int = 0, bath_efficiency: bool = False,
                   max_eff: int = 6, n_inert: int = 0, n_colliders: int = 8) -> Mechanism:
    """Seeded synthetic mechanism with ``ns`` species and ``nr`` reactions.

    ``n_inert`` species just before the bath gas take part in no reaction
    (like argon or helium in real models); they may still be colliders.
    """
    if ns < 3:
        raise ValueError("need at least 3 species")
    rng = np.random.Generator(np.random.PCG64(seed))
    bath = ns - 1
    comp = np.zeros((ns, 4), dtype=np.int64)
    comp[:bath] = _draw_compositions(rng, bath)
    comp[bath] = (0, 0, 0, 2)                   # N2-like bath gas
    W = comp @ np.array(ATOMIC_WEIGHTS)
    names = [f"S{k}" for k in range(bath)] + ["BATH"]
    a_lo = np.zeros((ns, 7))
    a_hi = np.zeros((ns, 7))
    for k in range(ns):
        atoms = int(comp[k].sum())
        h298 = 0.0 if k == bath else rng.uniform(-3.0e4, 3.0e4)
        s298 = rng.uniform(20.0, 40.0)
        a_lo[k], a_hi[k] = _fit_nasa(rng, atoms, h298, s298)
    tmid = np.full(ns, T_MID)

    # Zipf-like popularity over a random ranking of the non-bath species.
    n_react = bath - n_inert
    if n_react < 2:
        raise ValueError("too few reactive species")
    rank = rng.permutation(n_react) + 1
    pop = np.zeros(ns)
    pop[:n_react] = 1.0 / rank.astype(float) ** zipf
    pop /= pop.sum()

    allowed = np.zeros(ns, dtype=bool)
    allowed[:n_react] = True
    wprod = pop.copy()
    wprod[bath] = 1e-3 * pop[:n_react].min()
    allowed_b = allowed.copy()
    allowed_b[bath] = True
    pindex = _ProductIndex(comp, allowed, wprod)
    pindex_b = _ProductIndex(comp, allowed_b, wprod)

    # reaction type counts
    n_tb = int(round(mix.third_body * nr))
    n_fall = int(round(mix.falloff * nr))
    n_troe = n_fall // 2
    n_lind = n_fall - n_troe
    n_irr = int(round(mix.irreversible * nr))
    n_sri = int(round(mix.sri * nr))
    n_ca = int(round(mix.chem_act * nr))
    n_plog = int(round(mix.plog * nr))
    n_cheb = int(round(mix.cheb * nr))
    n_elem = nr - n_tb - n_fall - n_irr - n_sri - n_ca - n_plog - n_cheb
    if n_elem < 0:
        raise ValueError("type mix exceeds 100%")
    kinds = (["ELEM_REV"] * n_elem + ["ELEM_IRR"] * n_irr + ["THREEBODY"] * n_tb
             + ["LINDEMANN"] * n_lind + ["TROE"] * n_troe + ["SRI"] * n_sri
             + ["CA_" + FALLOFF_TYPES[t % 3] for t in range(n_ca)]
             + ["PLOG"] * n_plog + ["CHEB"] * n_cheb)
    kinds = [kinds[t] for t in rng.permutation(nr)]
    bath_slots = set(rng.choice(nr, size=min(bath_reactions, nr), replace=False).tolist()) \
        if bath_reactions else set()

    # Enhanced third bodies come from a small set of colliders (the most
    # popular species), as efficiencies in real mechanisms name the same few
    # species again and again.
    colliders = np.argsort(-pop[:bath], kind="stable")[:min(bath, max(max_eff, n_colliders))]
    if n_inert:
        colliders = np.concatenate([colliders[: max(1, len(colliders) - n_inert)],
                                    np.arange(n_react, bath)])

    seen = set()
    reactions: List[Reaction] = []
    for i, kind in enumerate(kinds):
        with_bath = i in bath_slots
        for _attempt in range(3000):
            pressure_dep = kind == "THREEBODY" or kind.replace("CA_", "") in FALLOFF_TYPES
            size = int(rng.choice([1, 2, 3], p=[0.15, 0.70, 0.15] if not pressure_dep
                                  else [0.3, 0.7, 0.0]))
            if with_bath:
                others = rng.choice(ns, size=size - 1, p=pop) if size > 1 else np.array([], dtype=int)
                reac_sp = [bath] + [int(s) for s in others]
            else:
                reac_sp = [int(s) for s in rng.choice(ns, size=size, p=pop)]
            reac = _multiset(reac_sp)
            if any(nu > 2 for _, nu in reac):
                continue
            key = comp[reac_sp].sum(axis=0)
            arr, wts = (pindex_b if with_bath else pindex).candidates(key)
            rset = np.array(sorted({s for s, _ in reac}), dtype=np.int64)
            keep = ~np.isin(arr, rset).any(axis=1)
            if pressure_dep:
                keep &= arr[:, 2] < 0
            if not np.any(keep):
                continue
            arr, wts = arr[keep], wts[keep]
            pick = arr[int(rng.choice(len(arr), p=wts / wts.sum()))]
            prod = _multiset([int(s) for s in pick if s >= 0])
            canon = (tuple(reac), tuple(prod))
            if canon in seen or (canon[1], canon[0]) in seen:
                continue
            seen.add(canon)
            break
        else:
            raise RuntimeError("could not draw a balanced reaction")
        lnA, b, th = _draw_arrhenius(rng)
        rx = Reaction(type="ELEM", rev=(kind != "ELEM_IRR"), reac=reac, prod=prod,
                      lnA=lnA, b=b, theta=th)
        if kind.startswith("CA_"):
            kind = kind[3:]
            rx.chemact = True
        if kind in ("THREEBODY",) + FALLOFF_TYPES:
            rx.type = kind
            m = int(rng.integers(1, max_eff + 1))
            chosen = rng.choice(colliders, size=min(m, len(colliders)), replace=False)
            rx.eff = [(int(s), float(rng.uniform(0.5, 5.0))) for s in sorted(chosen)]
            if bath_efficiency:
                rx.eff.append((bath, float(rng.uniform(0.5, 5.0))))
        if kind in FALLOFF_TYPES:
            rx.low = _draw_arrhenius(rng)
        if kind == "TROE":
            rx.troe = (float(rng.uniform(0.0, 1.0)), float(rng.uniform(100.0, 5000.0)),
                       float(rng.uniform(100.0, 5000.0)), float(rng.uniform(100.0, 5000.0)))
        if kind == "SRI":
            rx.sri = (float(rng.uniform(0.1, 2.0)), float(rng.uniform(100.0, 2000.0)),
                      float(rng.uniform(100.0, 2000.0)), float(rng.uniform(0.5, 2.0)),
                      float(rng.uniform(-0.5, 0.5)))
        if kind == "PLOG":
            rx.type = "PLOG"
            m_p = int(rng.integers(2, 6))
            lp = np.sort(rng.choice(np.linspace(-1.0, 2.5, 36), size=m_p, replace=False))
            rx.plog = [(float(ATM * 10.0 ** v), float(lnA + rng.uniform(-2.0, 2.0)),
                        float(b + rng.uniform(-0.5, 0.5)),
                        float(max(0.0, th + rng.uniform(-2000.0, 2000.0)))) for v in lp]
            rx.lnA, rx.b, rx.theta = 0.0, 0.0, 0.0
        if kind == "CHEB":
            rx.type = "CHEB"
            nt, npr = int(rng.integers(3, 7)), int(rng.integers(2, 5))
            coef = [[float(rng.normal(0.0, 0.3)) / (1 + t + q) for q in range(npr)] for t in range(nt)]
            coef[0][0] = float(rng.uniform(8.0, 13.0))
            coef[1][0] = float(rng.uniform(-3.0, 0.0))
            rx.cheb = ((290.0, 3000.0, 0.01 * ATM, 100.0 * ATM), coef)
            rx.lnA, rx.b, rx.theta = 0.0, 0.0, 0.0
        reactions.append(rx)
    return Mechanism(names=names, W=W, comp=comp, tmid=tmid, a_lo=a_lo, a_hi=a_hi,
                     reactions=reactions)


def workload_mechanism(name: str) -> Mechanism:
    w = WORKLOADS[name]
    return make_mechanism(w.ns, w.nr, w.mech_seed, mix=w.mix, zipf=w.zipf,
                          bath_reactions=w.bath_reactions, n_inert=w.n_inert)


# ----------------------------------------------------------------------------
# description file

def _g(x: float) -> str:
    return repr(float(x))


def dumps(m: Mechanism) -> str:
    lines = ["PJMECH 1", f"SPECIES {m.n_species}"]
    for k in range(m.n_species):
        c = m.comp[k]
        vals = [m.W[k], c[0], c[1], c[2], c[3], T_LOW, m.tmid[k], T_HIGH]
        lines.append(" ".join(["SP", str(k), m.names[k], _g(m.W[k])]
                              + [str(int(v)) for v in c]
                              + [_g(T_LOW), _g(m.tmid[k]), _g(T_HIGH)]
                              + [_g(v) for v in m.a_lo[k]] + [_g(v) for v in m.a_hi[k]]))
        del vals
    lines.append(f"REACTIONS {m.n_reactions}")
    for i, r in enumerate(m.reactions):
        tok = ["RX", str(i), r.type, "1" if r.rev else "0", str(len(r.reac))]
        for s, nu in r.reac:
            tok += [str(s), str(nu)]
        tok.append(str(len(r.prod)))
        for s, nu in r.prod:
            tok += [str(s), str(nu)]
        tok += [_g(r.lnA), _g(r.b), _g(r.theta)]
        if r.low is not None:
            tok += ["LOW"] + [_g(v) for v in r.low]
        if r.troe is not None:
            tok += ["TROE"] + [_g(v) for v in r.troe]
        if r.sri is not None:
            tok += ["SRI"] + [_g(v) for v in r.sri]
        if r.chemact:
            tok.append("CHEMACT")
        if r.plog is not None:
            tok += ["PLOG", str(len(r.plog))]
            for pt in r.plog:
                tok += [_g(v) for v in pt]
        if r.cheb is not None:
            rng_, coef = r.cheb
            tok += ["CHEB", str(len(coef)), str(len(coef[0]))] + [_g(v) for v in rng_]
            tok += [_g(v) for row in coef for v in row]
        if r.eff:
            tok += ["EFF", str(len(r.eff))]
            for s, a in r.eff:
                tok += [str(s), _g(a)]
        lines.append(" ".join(tok))
    lines.append("END")
    return "\n".join(lines) + "\n"


def write_mechanism(m: Mechanism, path: str) -> str:
    with open(path, "w") as f:
        f.write(dumps(m))
    return path


def loads(text: str) -> Mechanism:
    """Parse a description back into a :class:`Mechanism` (used by the tests
    of this module and by the generator's own round-trip check)."""
    tok = text.split()
    p = 0

    def nxt():
        nonlocal p
        p += 1
        return tok[p - 1]

    assert nxt() == "PJMECH" and nxt() == "1"
    assert nxt() == "SPECIES"
    ns = int(nxt())
    names, W, comp, tmid, a_lo, a_hi = [], [], [], [], [], []
    for _ in range(ns):
        assert nxt() == "SP"
        nxt()
        names.append(nxt())
        W.append(float(nxt()))
        comp.append([int(nxt()) for _ in range(4)])
        nxt()
        tmid.append(float(nxt()))
        nxt()
        a_lo.append([float(nxt()) for _ in range(7)])
        a_hi.append([float(nxt()) for _ in range(7)])
    assert nxt() == "REACTIONS"
    nr = int(nxt())
    rxs = []
    for _ in range(nr):
        assert nxt() == "RX"
        nxt()
        typ = nxt()
        rev = nxt() == "1"
        reac = [(int(nxt()), int(nxt())) for _ in range(int(nxt()))]
        prod = [(int(nxt()), int(nxt())) for _ in range(int(nxt()))]
        lnA, b, th = float(nxt()), float(nxt()), float(nxt())
        r = Reaction(typ, rev, reac, prod, lnA, b, th)
        while tok[p] in ("LOW", "TROE", "SRI", "CHEMACT", "PLOG", "CHEB", "EFF"):
            kw = nxt()
            if kw == "LOW":
                r.low = (float(nxt()), float(nxt()), float(nxt()))
            elif kw == "TROE":
                r.troe = (float(nxt()), float(nxt()), float(nxt()), float(nxt()))
            elif kw == "SRI":
                r.sri = tuple(float(nxt()) for _ in range(5))
            elif kw == "CHEMACT":
                r.chemact = True
            elif kw == "PLOG":
                r.plog = [tuple(float(nxt()) for _ in range(4)) for _ in range(int(nxt()))]
            elif kw == "CHEB":
                nt, npr = int(nxt()), int(nxt())
                rng_ = tuple(float(nxt()) for _ in range(4))
                r.cheb = (rng_, [[float(nxt()) for _ in range(npr)] for _ in range(nt)])
            else:
                r.eff = [(int(nxt()), float(nxt())) for _ in range(int(nxt()))]
        rxs.append(r)
    assert nxt() == "END"
    return Mechanism(names=names, W=np.array(W), comp=np.array(comp, dtype=np.int64),
                     tmid=np.array(tmid), a_lo=np.array(a_lo), a_hi=np.array(a_hi),
                     reactions=rxs)


# ----------------------------------------------------------------------------
# states

def make_states(m: Mechanism, n: int, seed: int, T_range=(600.0, 2200.0),
                P_range_atm=(1.0, 50.0), alpha: float = 0.5):
    """Seeded batch of ``n`` states.

    Returns ``dict(T, P, V, n)`` with ``n`` of shape (n, Ns) holding the moles
    of every species (the last column, the bath gas, is informative only: the
    state vector omits it).  Use :func:`pack_state` to build the library's
    input arrays.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    T = rng.uniform(T_range[0], T_range[1], size=n)
    P = rng.uniform(P_range_atm[0], P_range_atm[1], size=n) * ATM
    Y = rng.dirichlet(np.full(m.n_species, alpha), size=n) if n else np.zeros((0, m.n_species))
    X = Y / m.W[None, :]
    X /= X.sum(axis=1, keepdims=True)
    V = np.ones(n)
    ntot = P * V / (R_GAS * T)
    moles = X * ntot[:, None]
    return {"T": T, "P": P, "V": V, "n": moles}


def pack_state(st, form: str = "conp", layout: str = "C"):
    """(state, param) arrays for the given form and layout.

    CONP: state = (T, V, n_1..n_{Ns-1}), param = P.
    CONV: state = (T, P, n_1..n_{Ns-1}), param = V.
    Layout "C": state[s, i] (row-major, state-major);
    layout "F": state[i, s] (each variable over all states is contiguous).
    """
    T, P, V, moles = st["T"], st["P"], st["V"], st["n"]
    n = T.shape[0]
    ns = moles.shape[1]
    x = np.empty((n, ns + 1))
    x[:, 0] = T
    if form == "conp":
        x[:, 1] = V
        param = P.copy()
    elif form == "conv":
        x[:, 1] = P
        param = V.copy()
    else:
        raise ValueError(form)
    x[:, 2:] = moles[:, : ns - 1]
    if layout == "C":
        return np.ascontiguousarray(x), param
    if layout == "F":
        return np.ascontiguousarray(x.T), param
    raise ValueError(layout)


def workload_states(name: str, n: Optional[int] = None):
    w = WORKLOADS[name]
    m = workload_mechanism(name)
    return m, make_states(m, w.n_states if n is None else n, w.state_seed,
                          T_range=w.T_range, P_range_atm=w.P_range_atm)


def jacobian_pattern_density(nnz: int, N: int) -> float:
    return nnz / float(N * N)
