"""Seeded synthetic inputs: kinetic mechanisms and thermochemical states.

This module is the only code shared by the HIP path and the CPU oracle.  It
draws inputs; it evaluates none of the integrator's arithmetic (no rate
constants, no production rates, no Jacobian, no ROS4 step).

The paper integrates GRI-Mech 3.0 states from a partially-stirred-reactor
database and CFD cells (Sec. 3.1, Sec. 4); neither is available here, so
mechanisms of the same shape are synthesised:

* species are small C/H/O/N molecules (the last one is the inert bath gas N2,
  which the state vector omits, Sec. 2.1 eq. (state_vec), eq. (n_nsp));
* reactions are reversible, element-balanced, with stoichiometric
  coefficients 1-2 and at most three species per side; some are third-body,
  Lindemann or Troe falloff reactions;
* A ~ logU[1e8, 1e16] in mol-cm3-s units of the reaction order, b ~
  U[-1.5, 1.5], Ea ~ U[0, 200] kJ/mol; each reaction is oriented
  endothermic-forward and its Ea raised to at least the reaction enthalpy at
  298 K so that reverse rate constants stay bounded (reactions whose enthalpy
  exceeds 400 kJ/mol, or 600 kJ/mol for the third-body and falloff
  dissociations, are not drawn);
* thermodynamics are two-range NASA 7-coefficient fits of a smooth cp(T)
  curve, continuous in cp, h and s at T_mid = 1000 K.

Mechanism file format (text, one record per line, SI units: kmol, m3, s, K):

    CHEMMECH 1
    ELEMENTS <E> <sym_1> ... <sym_E>
    SPECIES <K>
    <name> <W kg/kmol> <E element counts> <T_mid> <a_lo 1..7> <a_hi 1..7>
    REACTIONS <Nr>
    <type> <nr> (<idx> <nu>)*nr <np> (<idx> <nu>)*np <lnA> <b> <theta>
           <neff> (<idx> <alpha>)*neff [<lnA0> <b0> <theta0>] [<a> <T3> <T1> <T2>]

type is E (elementary), T (third body), L (Lindemann falloff) or F (Troe
falloff).  Species indices are 0-based.  theta = Ea/R in K; A is in SI units
(kmol, m3, s) of the reaction order, the collider counting for T.  A falloff
line carries the high-pressure Arrhenius triple first and the low-pressure
triple after the efficiencies; Troe's T2 = 0 means the third term is absent.
Third-body efficiencies default to 1 for species not listed.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

R_J_MOL_K = 8.314462618          # J/(mol K)
P_ATM = 101325.0
ATOMIC_W = {"C": 12.011, "H": 1.008, "O": 15.999, "N": 14.007}
VALENCE = {"C": 4, "H": 1, "O": 2, "N": 3}
ATOM_HF = {"H": 218.0, "O": 249.2, "C": 716.7, "N": 472.7}   # kJ/mol, free atoms
T_MID = 1000.0


@dataclass
class Species:
    name: str
    comp: dict
    W: float
    lo: np.ndarray
    hi: np.ndarray
    hf298: float       # kJ/mol
    s298: float        # J/mol/K


@dataclass
class Reaction:
    kind: str                     # 'E', 'T', 'L', 'F'
    reac: list                    # [(idx, nu)]
    prod: list
    lnA: float
    b: float
    theta: float
    eff: list = field(default_factory=list)     # [(idx, alpha)]
    low: tuple | None = None      # (lnA0, b0, theta0)
    troe: tuple | None = None     # (a, T3, T1, T2)


@dataclass
class Mechanism:
    elements: list
    species: list
    reactions: list

    @property
    def n_species(self):
        return len(self.species)

    def index(self, name):
        for i, s in enumerate(self.species):
            if s.name == name:
                return i
        raise KeyError(name)

    def weights(self):
        return np.array([s.W for s in self.species])

    def write(self, path):
        with open(path, "w") as f:
            f.write(self.text())

    def text(self):
        r = repr
        out = ["CHEMMECH 1", "ELEMENTS %d %s" % (len(self.elements), " ".join(self.elements)),
               "SPECIES %d" % len(self.species)]
        for s in self.species:
            cnt = " ".join(str(s.comp.get(e, 0)) for e in self.elements)
            out.append("%s %s %s %s %s %s" % (s.name, r(float(s.W)), cnt, r(T_MID),
                                              " ".join(r(float(x)) for x in s.lo),
                                              " ".join(r(float(x)) for x in s.hi)))
        out.append("REACTIONS %d" % len(self.reactions))
        for q in self.reactions:
            parts = [q.kind, str(len(q.reac))]
            for i, nu in q.reac:
                parts += [str(i), str(nu)]
            parts.append(str(len(q.prod)))
            for i, nu in q.prod:
                parts += [str(i), str(nu)]
            parts += [r(float(q.lnA)), r(float(q.b)), r(float(q.theta)), str(len(q.eff))]
            for i, a in q.eff:
                parts += [str(i), r(float(a))]
            if q.kind in "LF":
                parts += [r(float(x)) for x in q.low]
            if q.kind == "F":
                parts += [r(float(x)) for x in q.troe]
            out.append(" ".join(parts))
        return "\n".join(out) + "\n"


# ----------------------------------------------------------------------------
# species pool and thermochemistry draws
# ----------------------------------------------------------------------------

def _formula(comp):
    s = ""
    for e in ("C", "H", "O", "N"):
        n = comp.get(e, 0)
        if n:
            s += e + (str(n) if n > 1 else "")
    return s


def _candidate_pool(elements, max_c, max_h, max_o, max_n):
    pool = []
    for c in range(0, max_c + 1 if "C" in elements else 1):
        for n in range(0, max_n + 1 if "N" in elements else 1):
            for o in range(0, max_o + 1):
                for h in range(0, max_h + 1):
                    atoms = c + h + o + n
                    if atoms == 0 or atoms > 10:
                        continue
                    # hydrogen cannot exceed what the heavy-atom skeleton can hold
                    if h > 2 * c + n + 2 + (2 if c == 0 and n == 0 else 0):
                        continue
                    comp = {k: v for k, v in (("C", c), ("H", h), ("O", o), ("N", n)) if v}
                    if comp == {"N": 2}:
                        continue            # the bath gas is appended separately
                    pool.append(comp)
    return pool


def _hf298(comp, rng, reference):
    """Heuristic formation enthalpy, kJ/mol (oxidation products low, radicals high)."""
    atoms = sum(comp.values())
    if atoms == 1:
        (e, _), = comp.items()
        return ATOM_HF[e]
    if reference:
        return 0.0
    nC, nH, nO, nN = (comp.get(e, 0) for e in ("C", "H", "O", "N"))
    vC, vO, vN = 4 * nC, 2 * nO, 3 * nN
    hr = nH
    nCH = min(hr, vC); hr -= nCH; vC -= nCH
    nOH = min(hr, vO); hr -= nOH; vO -= nOH
    nNH = min(hr, vN); hr -= nNH; vN -= nNH
    nCO = min(vC, vO)
    total_valence = 4 * nC + nH + 2 * nO + 3 * nN
    radical = total_valence % 2
    h = -(19.0 * nCH + 121.0 * nOH + 15.0 * nNH + 98.0 * nCO) + 160.0 * radical
    h += 45.0 * max(0, hr)      # dangling hydrogens
    return h + rng.normal(0.0, 12.0)


def _s298(comp, W, rng):
    atoms = sum(comp.values())
    if atoms == 1:
        return 110.0 + 1.0 * W + rng.uniform(-5, 5)
    return 90.0 + 20.0 * atoms + 1.0 * W + rng.uniform(-10, 10)


def _nasa7_fit(comp, hf, s298, rng):
    """Two-range NASA-7 coefficients of cp/R(T) = c_inf - (c_inf - c_0) exp(-T/tau)."""
    atoms = sum(comp.values())
    if atoms == 1:
        c0 = cinf = 2.5
    elif atoms == 2:
        c0, cinf = 3.5, 4.5
    else:
        c0, cinf = 4.0, 4.0 + (3 * atoms - 6)
    tau = rng.uniform(500.0, 1500.0)
    cp = lambda T: cinf - (cinf - c0) * np.exp(-T / tau)
    Tl = np.linspace(300.0, T_MID, 141)
    Th = np.linspace(T_MID, 3500.0, 251)
    Pl = np.polynomial.Polynomial.fit(Tl, cp(Tl), 4, domain=[-1, 1], window=[-1, 1])
    lo = np.array(Pl.coef, dtype=float)
    # high range: cp continuous at T_mid (eliminate the constant term)
    cp_mid = np.polynomial.Polynomial(lo)(T_MID)
    X = np.stack([Th - T_MID, Th ** 2 - T_MID ** 2, Th ** 3 - T_MID ** 3, Th ** 4 - T_MID ** 4], 1)
    coef, *_ = np.linalg.lstsq(X, cp(Th) - cp_mid, rcond=None)
    a1 = cp_mid - (coef[0] * T_MID + coef[1] * T_MID ** 2 + coef[2] * T_MID ** 3 + coef[3] * T_MID ** 4)
    hi = np.array([a1, *coef], dtype=float)

    def H_over_R(c, T):          # integral of cp/R dT (constant dropped)
        return np.polynomial.Polynomial(c).integ()(T)

    def S_over_R(c, T):          # integral of cp/(R T) dT (constant dropped)
        return c[0] * np.log(T) + np.polynomial.Polynomial(c[1:]).integ()(T)

    a6_lo = hf * 1000.0 / R_J_MOL_K - H_over_R(lo, 298.15)
    a7_lo = s298 / R_J_MOL_K - S_over_R(lo, 298.15)
    a6_hi = H_over_R(lo, T_MID) + a6_lo - H_over_R(hi, T_MID)
    a7_hi = S_over_R(lo, T_MID) + a7_lo - S_over_R(hi, T_MID)
    return np.r_[lo, a6_lo, a7_lo], np.r_[hi, a6_hi, a7_hi]


# ----------------------------------------------------------------------------
# mechanism generator
# ----------------------------------------------------------------------------

def _key(comp, elements):
    return tuple(comp.get(e, 0) for e in elements)


def generate_mechanism(n_species, n_reactions, n_third_body, n_falloff, troe, elements,
                       max_c, seed, must_have=(), core=()):
    """Draw an element-balanced reversible mechanism.

    n_falloff reactions are Troe if ``troe`` else Lindemann.  The last species
    is N2 and is inert (collider only).  ``core`` lists reactions by species
    names, ``(kind, reactants, products)``, that the mechanism must contain
    (drawn first, with rate parameters from the same distributions as the
    rest; they count towards n_reactions and the third-body/falloff totals).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    pool = _candidate_pool(elements, max_c, max_h=2 * max_c + 4 if max_c else 4,
                           max_o=3 if max_c >= 3 else 2, max_n=1 if "N" in elements else 0)
    chosen = []
    for f in must_have:
        comp = _parse_formula(f)
        if comp not in chosen:
            chosen.append(comp)
    rest = [c for c in pool if c not in chosen]
    # favour small molecules, like real mechanisms
    w = np.array([1.0 / (1.0 + sum(c.values())) ** 1.5 for c in rest])
    pick = rng.choice(len(rest), size=n_species - 1 - len(chosen), replace=False, p=w / w.sum())
    chosen += [rest[i] for i in sorted(pick)]
    chosen.append({"N": 2})
    species = []
    for comp in chosen:
        W = sum(ATOMIC_W[e] * n for e, n in comp.items())
        reference = comp in ({"H": 2}, {"O": 2}, {"N": 2})
        hf = _hf298(comp, rng, reference)
        s = _s298(comp, W, rng)
        lo, hi = _nasa7_fit(comp, hf, s, rng)
        species.append(Species(_formula(comp), comp, W, lo, hi, hf, s))
    K = len(species)
    active = K - 1           # the bath gas never reacts
    keys = [_key(s.comp, elements) for s in species]
    hf = np.array([s.hf298 for s in species])

    singles = {}
    pairs = {}
    triples = {}
    for i in range(active):
        singles.setdefault(keys[i], []).append(((i, 1),))
        for j in range(i, active):
            k = tuple(a + b for a, b in zip(keys[i], keys[j]))
            side = ((i, 2),) if i == j else ((i, 1), (j, 1))
            pairs.setdefault(k, []).append(side)
            for l in range(j, active):
                if l == i:
                    continue            # no species with coefficient 3
                k3 = tuple(a + b for a, b in zip(k, keys[l]))
                if l == j:
                    side3 = ((i, 1), (j, 2))
                elif i == j:
                    side3 = ((i, 2), (l, 1))
                else:
                    side3 = ((i, 1), (j, 1), (l, 1))
                triples.setdefault(k3, []).append(side3)

    def dH(reac, prod):
        return sum(nu * hf[i] for i, nu in prod) - sum(nu * hf[i] for i, nu in reac)

    def order(side):
        return sum(nu for _, nu in side)

    seen = set()
    reactions = []
    uses = np.zeros(active, int)
    kinds = ["T"] * n_third_body + ["F" if troe else "L"] * n_falloff
    kinds += ["E"] * (n_reactions - len(kinds))

    def finish(kind, reac, prod, h):
        """Rate parameters of a reaction oriented endothermic-forward (enthalpy h)."""
        for x, _ in reac + prod:
            uses[x] += 1
        Ea = max(rng.uniform(0.0, 200.0), h)            # kJ/mol
        theta = Ea * 1000.0 / R_J_MOL_K
        b = rng.uniform(-1.5, 1.5)
        A_cgs = 10.0 ** rng.uniform(8.0, 16.0)
        ordr = order(reac) + (1 if kind == "T" else 0)
        lnA = math.log(A_cgs) + (ordr - 1) * math.log(1e-3)
        eff = []
        low = None
        tr = None
        if kind != "E":
            ne = int(rng.integers(0, 4))
            for s_ in rng.choice(K, size=ne, replace=False):
                eff.append((int(s_), float(rng.uniform(0.4, 6.0))))
            eff.sort()
        if kind in "LF":
            A0_cgs = A_cgs * 10.0 ** rng.uniform(3.0, 7.0)
            lnA0 = math.log(A0_cgs) + order(reac) * math.log(1e-3)
            low = (lnA0, rng.uniform(-1.5, 1.5), rng.uniform(0.0, theta))
        if kind == "F":
            a = rng.uniform(0.1, 0.9)
            T3 = math.exp(rng.uniform(math.log(30.0), math.log(1000.0)))
            T1 = math.exp(rng.uniform(math.log(500.0), math.log(5000.0)))
            T2 = math.exp(rng.uniform(math.log(1000.0), math.log(1e4))) if rng.random() < 0.5 else 0.0
            tr = (a, T3, T1, T2)
        reactions.append(Reaction(kind, list(reac), list(prod), lnA, b, theta, eff, low, tr))

    names = [_formula(c) for c in chosen]
    for kind, rs, ps in core:
        if kind != "E":
            kinds.remove("F" if (kind in "LF" and troe) else ("L" if kind in "LF" else "T"))
        else:
            kinds.remove("E")
        side = lambda xs: tuple(sorted((names.index(_formula(_parse_formula(n_))), c_) for n_, c_ in
                                       {n_: xs.count(n_) for n_ in xs}.items()))
        reac, prod = side(rs), side(ps)
        assert _key_sum(reac, keys) == _key_sum(prod, keys), (rs, ps)
        kind = ("F" if troe else "L") if kind in "LF" else kind
        seen.add((tuple(sorted(reac)), tuple(sorted(prod))))
        h = dH(reac, prod)
        if h < 0:
            reac, prod, h = prod, reac, -h
        finish(kind, reac, prod, h)
    attempts = 0
    while len(reactions) < n_reactions:
        attempts += 1
        if attempts > 200000:
            raise RuntimeError("could not draw enough reactions")
        kind = kinds[len(reactions) - len(core)]
        if kind == "E":
            # bimolecular exchange A + B = C + D, seeded from a rarely used species
            if rng.random() < 0.5:
                i = int(np.argmin(uses + rng.random(active)))
            else:
                i = int(rng.integers(active))
            j = int(rng.integers(active))
            a, b = min(i, j), max(i, j)
            reac = ((a, 2),) if a == b else ((a, 1), (b, 1))
            k = tuple(x + y for x, y in zip(keys[a], keys[b]))
            cands = [p for p in pairs.get(k, []) if p != reac]
            r_ = rng.random()
            if r_ < 0.15:
                cands += [p for p in singles.get(k, [])]
            elif r_ < 0.25:
                cands += [p for p in triples.get(k, [])]
        else:
            # association / dissociation A + B (+M) = AB (+M)
            cands = []
            i = int(rng.integers(active))
            if sum(species[i].comp.values()) < 2:
                continue
            reac = ((i, 1),)
            cands = [p for p in pairs.get(keys[i], [])]
        if not cands:
            continue
        prod = cands[int(rng.integers(len(cands)))]
        if set(x for x, _ in prod) & set(x for x, _ in reac):
            continue
        sig = (tuple(sorted(reac)), tuple(sorted(prod)))
        if sig in seen or (sig[1], sig[0]) in seen:
            continue
        h = dH(reac, prod)
        if h < 0:
            reac, prod, h = prod, reac, -h
        # bond fissions (the third-body and falloff dissociations) keep their
        # larger enthalpy
        if h > (400.0 if kind == "E" else 600.0):
            continue
        seen.add(sig)
        finish(kind, reac, prod, h)
    order_ix = rng.permutation(len(reactions))
    reactions = [reactions[i] for i in order_ix]
    return Mechanism(list(elements), species, reactions)


def _key_sum(side, keys):
    return tuple(sum(nu * keys[i][e] for i, nu in side) for e in range(len(keys[0])))


def _parse_formula(f):
    comp, i = {}, 0
    while i < len(f):
        e = f[i]
        i += 1
        n = ""
        while i < len(f) and f[i].isdigit():
            n += f[i]
            i += 1
        comp[e] = comp.get(e, 0) + (int(n) if n else 1)
    return comp


# ----------------------------------------------------------------------------
# the workload mechanisms
# ----------------------------------------------------------------------------

H2O2_SPECIES = ("H2", "H", "O", "O2", "OH", "H2O", "HO2", "NO", "NO2")
CH4_MUST = ("H2", "H", "O", "O2", "OH", "H2O", "HO2", "H2O2", "C", "CH", "CH2", "CH3", "CH4",
            "CO", "CO2", "CHO", "CH2O", "CH3O", "CH4O", "C2H2", "C2H4", "C2H6", "NO", "N",
            "HN", "NO2", "N2O")


def mech_small(seed=101):
    """10 species (H, O, N; N2 inert, last), 25 reactions: 4 third-body, 2 Lindemann."""
    return generate_mechanism(10, 25, 4, 2, False, ["H", "O", "N"], 0, seed,
                              must_have=H2O2_SPECIES)


def mech_ch4(seed=102):
    """53 species (C, H, O, N; at most C3), 325 reactions: 30 third-body, 25 Troe."""
    return generate_mechanism(53, 325, 30, 25, True, ["C", "H", "O", "N"], 3, seed,
                              must_have=CH4_MUST)


# The fuel's own chemistry, present in every hydrocarbon mechanism: unimolecular
# decomposition, hydrogen abstraction by O2 and by the radical pool, the
# H + O2 branching step and the main oxidation path of the methyl radical.
FUEL_CORE = (
    ("F", ["CH4"], ["CH3", "H"]),
    ("E", ["CH4", "O2"], ["CH3", "HO2"]),
    ("E", ["CH4", "H"], ["CH3", "H2"]),
    ("E", ["CH4", "O"], ["CH3", "OH"]),
    ("E", ["CH4", "OH"], ["CH3", "H2O"]),
    ("E", ["CH4", "HO2"], ["CH3", "H2O2"]),
    ("E", ["H", "O2"], ["O", "OH"]),
    ("E", ["CH3", "O2"], ["CH3O", "O"]),
    ("E", ["CH3", "HO2"], ["CH3O", "OH"]),
    ("E", ["CH2O", "OH"], ["CHO", "H2O"]),
    ("E", ["CHO", "O2"], ["CO", "HO2"]),
    ("E", ["CO", "OH"], ["CO2", "H"]),
)


def mech_large(seed=104):
    """111 species (C, H, O, N; at most C4), 784 reactions: 60 third-body, 40 Troe,
    with the fuel core (FUEL_CORE).  Without it the draw for this seed holds a
    single route out of the fuel/air mixture (CH4 (+M) = H2 + CH2, with a rate
    constant five orders below the CH4-shaped mechanism's), and mixtures at
    1,600 K take one step per 1e-5 s: chemically inert."""
    return generate_mechanism(111, 784, 60, 40, True, ["C", "H", "O", "N"], 4, seed,
                              must_have=CH4_MUST, core=FUEL_CORE)


def mech_n30(seed=106):
    """30 species (C, H, O, N; at most C2), 180 reactions: 16 third-body, 12 Troe."""
    return generate_mechanism(30, 180, 16, 12, True, ["C", "H", "O", "N"], 2, seed,
                              must_have=CH4_MUST)


def mech_n45(seed=107):
    """45 species (C, H, O, N; at most C3), 260 reactions: 24 third-body, 18 Troe."""
    return generate_mechanism(45, 260, 24, 18, True, ["C", "H", "O", "N"], 3, seed,
                              must_have=CH4_MUST)


def mech_n62(seed=108):
    """62 species (C, H, O, N; at most C3), 380 reactions: 34 third-body, 28 Troe."""
    return generate_mechanism(62, 380, 34, 28, True, ["C", "H", "O", "N"], 3, seed,
                              must_have=CH4_MUST)


def mech_n15(seed=109):
    """15 species (C, H, O, N; C1 only), 60 reactions: 6 third-body, 4 Troe
    (state size 16: exactly the rows of the smallest one-wavefront-per-cell
    kernel)."""
    return generate_mechanism(15, 60, 6, 4, True, ["C", "H", "O", "N"], 1, seed,
                              must_have=("H2", "H", "O", "O2", "OH", "H2O", "HO2", "CH3", "CH4",
                                         "CO", "CO2", "CHO"))


def mech_n55(seed=110):
    """55 species (C, H, O, N; at most C3), 330 reactions: 30 third-body, 24 Troe
    (state size 56: exactly the rows of the 56-row kernel)."""
    return generate_mechanism(55, 330, 30, 24, True, ["C", "H", "O", "N"], 3, seed,
                              must_have=CH4_MUST)


def mech_n63(seed=111):
    """63 species (C, H, O, N; at most C3), 385 reactions: 34 third-body, 28 Troe
    (state size 64: one row per lane of the wavefront)."""
    return generate_mechanism(63, 385, 34, 28, True, ["C", "H", "O", "N"], 3, seed,
                              must_have=CH4_MUST)


def mech_n127(seed=119):
    """127 species (C, H, O, N; at most C4), 880 reactions: 66 third-body, 44 Troe,
    with the fuel core (state size 128: the largest state of the
    four-wavefront kernels, one row per lane in both halves).  The seed is one
    whose mixtures react within 1e-5 s (up to ~100 steps); several nearby
    draws take a single step there."""
    return generate_mechanism(127, 880, 66, 44, True, ["C", "H", "O", "N"], 4, seed,
                              must_have=CH4_MUST, core=FUEL_CORE)


MECHS = {"small": mech_small, "ch4": mech_ch4, "large": mech_large,
         "n15": mech_n15, "n30": mech_n30, "n45": mech_n45, "n55": mech_n55,
         "n62": mech_n62, "n63": mech_n63, "n127": mech_n127}


def mechanism_file(name, directory):
    """Write mechanism ``name`` to ``directory`` (cached by content) and return the path."""
    m = MECHS[name]()
    path = os.path.join(directory, "mech_%s.txt" % name)
    text = m.text()
    if not (os.path.exists(path) and open(path).read() == text):
        os.makedirs(directory, exist_ok=True)
        tmp = path + ".%d.tmp" % os.getpid()
        with open(tmp, "w") as f:
            f.write(text)
        os.replace(tmp, path)
    return path, m


# ----------------------------------------------------------------------------
# states
# ----------------------------------------------------------------------------

def _mix(mech, Z):
    """Mass fractions of fuel (CH4) / air (O2 0.233, N2 0.767) mixed at mixture fraction Z."""
    K = mech.n_species
    Y = np.zeros((K, Z.size))
    Y[mech.index("CH4")] = Z
    Y[mech.index("O2")] = (1.0 - Z) * 0.233
    Y[K - 1] = (1.0 - Z) * 0.767
    return Y


def z_stoich(mech):
    W = mech.weights()
    w_f, w_o = W[mech.index("CH4")], W[mech.index("O2")]
    # CH4 + 2 O2: mass of fuel per mass of air at stoichiometry
    r = w_f / (2 * w_o / 0.233)
    return r / (1.0 + r)


def _burnt(mech, Z):
    """Complete-combustion products of the fuel/air mixture at Z (CO2, H2O, leftover O2 or CH4)."""
    W = mech.weights()
    K = mech.n_species
    iF, iO, iC, iW = (mech.index(s) for s in ("CH4", "O2", "CO2", "H2O"))
    nF = Z / W[iF]
    nO = (1 - Z) * 0.233 / W[iO]
    burn = np.minimum(nF, nO / 2.0)
    Y = np.zeros((K, Z.size))
    Y[iF] = (nF - burn) * W[iF]
    Y[iO] = (nO - 2 * burn) * W[iO]
    Y[iC] = burn * W[iC]
    Y[iW] = 2 * burn * W[iW]
    Y[K - 1] = (1 - Z) * 0.767
    return Y / Y.sum(0, keepdims=True)


def states_small(mech, n=256, seed=201):
    """T ~ U[900, 2000] K, P = 1 atm, Y ~ Dirichlet(1) over all species."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = rng.uniform(900.0, 2000.0, n)
    P = np.full(n, P_ATM)
    Y = rng.dirichlet(np.ones(mech.n_species), n).T.copy()
    Y /= Y.sum(0, keepdims=True)
    return T, P, np.ascontiguousarray(Y)


def states_mixing(mech, n, seed):
    """CH4 (300 K) / air (800 K) mixing states: Z ~ Beta(2, 5), P ~ U[1, 5] atm.

    T is the linear mix of the stream temperatures plus N(0, 200^2) K,
    clipped to [300, 2400] K.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Z = rng.beta(2.0, 5.0, n)
    P = rng.uniform(1.0, 5.0, n) * P_ATM
    T = Z * 300.0 + (1.0 - Z) * 800.0 + rng.normal(0.0, 200.0, n)
    T = np.clip(T, 300.0, 2400.0)
    return T, P, np.ascontiguousarray(_mix(mech, Z))


def states_batching(mech, n, seed=203):
    """85 % cold (T < 800 K), 10 % near ignition (stoichiometric, 1100-1400 K), 5 % burnt gas."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_ign = int(round(0.10 * n))
    n_burnt = int(round(0.05 * n))
    n_cold = n - n_ign - n_burnt
    P = rng.uniform(1.0, 5.0, n) * P_ATM
    Zc = rng.beta(2.0, 5.0, n_cold)
    Tc = rng.uniform(300.0, 800.0, n_cold)
    Zi = np.full(n_ign, z_stoich(mech))
    Ti = rng.uniform(1100.0, 1400.0, n_ign)
    Zb = rng.uniform(0.03, 0.08, n_burnt)
    Tb = rng.uniform(1800.0, 2300.0, n_burnt)
    T = np.concatenate([Tc, Ti, Tb])
    Y = np.concatenate([_mix(mech, Zc), _mix(mech, Zi), _burnt(mech, Zb)], axis=1)
    kind = np.concatenate([np.zeros(n_cold, np.int8), np.ones(n_ign, np.int8), np.full(n_burnt, 2, np.int8)])
    perm = rng.permutation(n)
    return T[perm], P, np.ascontiguousarray(Y[:, perm]), kind[perm]


def loss_weights(mech, seed=305):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, 1.0, mech.n_species)
