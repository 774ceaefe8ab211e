"""Seeded synthetic reaction networks.

A network is a list of species, each with integer element counts and a charge,
and a list of reactions.  Every reaction has one or two reactants, one to three
products, a rate-law type and three parameters (alpha, beta, gamma).  The rate
laws themselves (Kooij-Arrhenius two-body, direct cosmic-ray ionisation, and
photo-reactions attenuated by visual extinction; paper Sec. 2 and App. B.1)
are evaluated by the solver and by the oracle, never here.

Products are drawn uniformly among all multisets of one to three species whose
element and charge totals equal those of the reactants and which differ from
the reactant multiset; this is rejection sampling from a uniform multiset
proposal conditioned on conservation.  Every reaction therefore conserves each
element and charge exactly (integer arithmetic).

Two families are built:

* the 12-species {H, C, O} + charge network (30 two-body ion-neutral or
  neutral-neutral reactions and 10 cosmic-ray reactions);
* large networks over {H, He, C, N, O, S} + charge (e.g. 200 species / 2500
  reactions or 500 species / 6000 reactions) with an 80/10/10 mix of two-body,
  cosmic-ray and photo reactions.
"""
from __future__ import annotations

import dataclasses
import io
import collections
import itertools

import numpy as np

ELEMENTS = ("H", "He", "C", "N", "O", "S")
N_ELEM = len(ELEMENTS)

TWO_BODY = 0
COSMIC_RAY = 1
PHOTO = 2
CR_PHOTON = 3   # photoreaction by cosmic-ray-induced photons
RTYPE_NAMES = {TWO_BODY: "two_body", COSMIC_RAY: "cosmic_ray", PHOTO: "photo", CR_PHOTON: "cr_photon"}

# packed composition key: one base-32 digit per element, one for charge+1 per species
_BASE = 32
_QDIG = _BASE ** N_ELEM


@dataclasses.dataclass
class Network:
    name: str
    species: list
    comp: np.ndarray       # (S, 6) int64 element counts
    charge: np.ndarray     # (S,) int64
    rtype: np.ndarray      # (R,) int32, TWO_BODY / COSMIC_RAY / PHOTO / CR_PHOTON
    reactants: np.ndarray  # (R, 2) int32, ascending, -1 padded
    products: np.ndarray   # (R, 3) int32, ascending, -1 padded at the end
    alpha: np.ndarray      # (R,) float64
    beta: np.ndarray       # (R,) float64
    gamma: np.ndarray      # (R,) float64
    albedo: float = 0.0    # dust albedo of the cosmic-ray-induced photon rate

    @property
    def n_species(self) -> int:
        return len(self.species)

    @property
    def n_reactions(self) -> int:
        return int(self.rtype.shape[0])

    def index(self, name: str) -> int:
        return self.species.index(name)

    def conservation_matrix(self) -> np.ndarray:
        """(E+1, S) integer matrix: element counts, then charge, per species."""
        return np.vstack([self.comp.T, self.charge[None, :]]).astype(np.int64)

    def to_text(self) -> str:
        out = io.StringIO()
        out.write("astrobdf-network 1\n")
        out.write(f"name {self.name}\n")
        if self.albedo != 0.0 or (np.asarray(self.rtype) == CR_PHOTON).any():
            out.write(f"albedo {float(self.albedo)!r}\n")
        out.write(f"elements {N_ELEM} {' '.join(ELEMENTS)}\n")
        out.write(f"species {self.n_species}\n")
        for i, s in enumerate(self.species):
            counts = " ".join(str(int(v)) for v in self.comp[i])
            out.write(f"{i} {s} {int(self.charge[i])} {counts}\n")
        out.write(f"reactions {self.n_reactions}\n")
        for r in range(self.n_reactions):
            re = [int(v) for v in self.reactants[r]]
            pr = [int(v) for v in self.products[r]]
            nr = sum(v >= 0 for v in re)
            npr = sum(v >= 0 for v in pr)
            out.write(
                f"{r} {int(self.rtype[r])} {nr} {re[0]} {re[1]} {npr} {pr[0]} {pr[1]} {pr[2]} "
                f"{float(self.alpha[r])!r} {float(self.beta[r])!r} {float(self.gamma[r])!r}\n"
            )
        out.write("end\n")
        return out.getvalue()


def write_network(net: Network, path) -> None:
    with open(path, "w") as fh:
        fh.write(net.to_text())


def species_name(comp, charge) -> str:
    """Hill-order formula (C, H, then the rest alphabetically) plus a charge mark."""
    if sum(comp) == 0:
        return "e-"
    cnt = dict(zip(ELEMENTS, comp))
    order = ["C", "H"] + sorted(e for e in ELEMENTS if e not in ("C", "H"))
    s = ""
    for e in order:
        n = cnt[e]
        if n == 1:
            s += e
        elif n > 1:
            s += f"{e}{n}"
    if charge > 0:
        s += "+" * charge
    elif charge < 0:
        s += "-" * (-charge)
    return s


def _comp(**kw):
    return tuple(int(kw.get(e, 0)) for e in ELEMENTS)


class _ProductTable:
    """Enumerates conserving product multisets of size 1..3 for a network's species."""

    def __init__(self, comp: np.ndarray, charge: np.ndarray):
        self.S = comp.shape[0]
        w = _BASE ** np.arange(N_ELEM, dtype=np.int64)
        self.key = comp.astype(np.int64) @ w + (charge.astype(np.int64) + 1) * _QDIG
        a, b = np.triu_indices(self.S)
        pk = self.key[a] + self.key[b]
        order = np.argsort(pk, kind="stable")
        self.pa, self.pb, self.pk = a[order], b[order], pk[order]
        self.w = w

    def target(self, comp_tot: np.ndarray, charge_tot: int, m: int) -> np.int64:
        return np.int64(int(comp_tot @ self.w) + (int(charge_tot) + m) * _QDIG)

    def candidates(self, comp_tot, charge_tot) -> list:
        out = []
        t1 = self.target(comp_tot, charge_tot, 1)
        for s in np.nonzero(self.key == t1)[0]:
            out.append((int(s),))
        t2 = self.target(comp_tot, charge_tot, 2)
        lo = int(np.searchsorted(self.pk, t2, side="left"))
        hi = int(np.searchsorted(self.pk, t2, side="right"))
        for i in range(lo, hi):
            out.append((int(self.pa[i]), int(self.pb[i])))
        t3 = self.target(comp_tot, charge_tot, 3)
        need = t3 - self.key
        lo = np.searchsorted(self.pk, need, side="left")
        hi = np.searchsorted(self.pk, need, side="right")
        cnt = hi - lo
        tot = int(cnt.sum())
        if tot:
            cs = np.repeat(np.arange(self.S), cnt)
            start = np.repeat(lo, cnt)
            offs = np.arange(tot) - np.repeat(np.cumsum(cnt) - cnt, cnt)
            idx = start + offs
            keep = self.pb[idx] <= cs
            for a, b, c in zip(self.pa[idx][keep], self.pb[idx][keep], cs[keep]):
                out.append((int(a), int(b), int(c)))
        out.sort(key=lambda t: (len(t), t))
        return out


def _loguniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


class _Builder:
    def __init__(self, name, species, comp, charge, rng):
        self.name = name
        self.species = list(species)
        self.comp = np.asarray(comp, dtype=np.int64)
        self.charge = np.asarray(charge, dtype=np.int64)
        self.rng = rng
        self.table = _ProductTable(self.comp, self.charge)
        self.rows = []          # (type, reactants tuple, products tuple, alpha, beta, gamma)
        self.seen = set()

    def conserving_products(self, reactants):
        ct = self.comp[list(reactants)].sum(axis=0)
        qt = int(self.charge[list(reactants)].sum())
        cands = self.table.candidates(ct, qt)
        rs = tuple(sorted(reactants))
        return [p for p in cands if p != rs]

    def add(self, rtype, reactants, products, alpha, beta, gamma):
        key = (tuple(sorted(reactants)), tuple(sorted(products)))
        if key in self.seen:
            return False
        self.seen.add(key)
        self.rows.append((rtype, key[0], key[1], float(alpha), float(beta), float(gamma)))
        return True

    def two_body(self, a, b):
        """One two-body reaction of the pair (a, b) with products drawn uniformly among
        the conserving multisets; False if none exists or it duplicates a reaction."""
        cands = self.conserving_products((a, b))
        if not cands:
            return False
        prod = cands[self.rng.integers(len(cands))]
        alpha = _loguniform(self.rng, 1e-12, 1e-9)
        beta = self.rng.uniform(-1.0, 1.0)
        gamma = self.rng.uniform(0.0, 200.0)
        return self.add(TWO_BODY, (a, b), prod, alpha, beta, gamma)

    def single(self, rtype, a, need_electron, e_idx):
        cands = self.conserving_products((a,))
        if need_electron:
            cands = [p for p in cands if e_idx in p]
        if not cands:
            return False
        prod = cands[self.rng.integers(len(cands))]
        if rtype == COSMIC_RAY:
            alpha, beta, gamma = _loguniform(self.rng, 0.1, 10.0), 0.0, 0.0
        else:
            alpha = _loguniform(self.rng, 1e-11, 1e-9)
            beta, gamma = 0.0, self.rng.uniform(0.5, 3.5)
        return self.add(rtype, (a,), prod, alpha, beta, gamma)

    def draw_two_body(self, pairs, count):
        made = 0
        while made < count:
            a, b = pairs[self.rng.integers(len(pairs))]
            if self.two_body(a, b):
                made += 1

    def draw_single(self, rtype, reactant_pool, count, need_electron, e_idx):
        made = 0
        tries = 0
        while made < count:
            tries += 1
            if tries > 200 * count + 1000:
                raise RuntimeError("could not draw enough single-reactant reactions")
            a = reactant_pool[self.rng.integers(len(reactant_pool))]
            cands = self.conserving_products((a,))
            if need_electron:
                cands = [p for p in cands if e_idx in p]
            if not cands:
                continue
            prod = cands[self.rng.integers(len(cands))]
            if rtype == COSMIC_RAY:
                alpha, beta, gamma = _loguniform(self.rng, 0.1, 10.0), 0.0, 0.0
            else:
                alpha = _loguniform(self.rng, 1e-11, 1e-9)
                beta, gamma = 0.0, self.rng.uniform(0.5, 3.5)
            if self.add(rtype, (a,), prod, alpha, beta, gamma):
                made += 1

    def grow(self, reach, kinds, allowed_pair, single_ok, e_idx):
        """Draws reactions of the given kinds, in order, with every reactant taken
        from the species already reachable from the initial state (`reach`,
        updated in place with each reaction's products), so that the network is
        connected to the initial abundances as a real chemical network is.
        Two-body pairs are uniform over the allowed unordered pairs of reachable
        species; single-reactant reactions take a uniform reachable species.
        kinds: sequence of TWO_BODY / COSMIC_RAY / PHOTO."""
        n = len(self.species)
        queue = collections.deque(kinds)
        stalled = 0
        while queue:
            kind = queue.popleft()
            for _ in range(3000 if not reach.all() else 300000):
                pool = np.flatnonzero(reach)
                if kind == TWO_BODY:
                    a, b = sorted(int(v) for v in pool[self.rng.integers(len(pool), size=2)])
                    # uniform over unordered pairs: a distinct pair arises from two orders
                    if a != b and self.rng.random() < 0.5:
                        continue
                    if not allowed_pair(a, b) or not self.two_body(a, b):
                        continue
                else:
                    a = int(pool[self.rng.integers(len(pool))])
                    if not single_ok(kind, a) or not self.single(kind, a, kind == COSMIC_RAY, e_idx):
                        continue
                for p in self.rows[-1][2]:
                    reach[p] = True
                stalled = 0
                break
            else:
                # nothing new of this kind among the reachable species yet: later
                queue.append(kind)
                stalled += 1
                if stalled > len(queue):
                    if reach.all():
                        raise RuntimeError("could not draw the remaining reactions")
                    # the reachable part is exhausted: the rest of the reactions
                    # are drawn among all species
                    reach[:] = True
                    stalled = 0
        return int(reach[:n].sum())

    def build(self) -> Network:
        R = len(self.rows)
        rtype = np.zeros(R, np.int32)
        rea = -np.ones((R, 2), np.int32)
        pro = -np.ones((R, 3), np.int32)
        al, be, ga = np.zeros(R), np.zeros(R), np.zeros(R)
        for i, (t, rs, ps, a, b, g) in enumerate(self.rows):
            rtype[i] = t
            rea[i, : len(rs)] = rs
            pro[i, : len(ps)] = ps
            al[i], be[i], ga[i] = a, b, g
        return Network(self.name, self.species, self.comp, self.charge, rtype, rea, pro, al, be, ga)


# ---------------------------------------------------------------------------
# 12-species {H, C, O} network
# ---------------------------------------------------------------------------
SMALL_SPECIES = [
    ("e-", _comp(), -1),
    ("H", _comp(H=1), 0),
    ("H2", _comp(H=2), 0),
    ("H+", _comp(H=1), 1),
    ("H2+", _comp(H=2), 1),
    ("H3+", _comp(H=3), 1),
    ("C", _comp(C=1), 0),
    ("C+", _comp(C=1), 1),
    ("O", _comp(O=1), 0),
    ("CO", _comp(C=1, O=1), 0),
    ("CO+", _comp(C=1, O=1), 1),
    ("HCO+", _comp(H=1, C=1, O=1), 1),
]


def small_network(seed: int = 1, n_two_body: int = 30, n_cr: int = 10) -> Network:
    """12 species over {H, C, O} + charge; ion-neutral / neutral-neutral two-body
    reactions (no electron reactant, no ion-ion pair) and cosmic-ray reactions.

    The cosmic-ray set holds every neutral single-reactant reaction that frees an
    electron, topped up with seeded draws from the other conserving
    single-reactant reactions."""
    rng = np.random.default_rng(seed)
    names = [s[0] for s in SMALL_SPECIES]
    comp = [s[1] for s in SMALL_SPECIES]
    charge = [s[2] for s in SMALL_SPECIES]
    bld = _Builder(f"small-{seed}", names, comp, charge, rng)
    e = 0
    non_e = [i for i in range(len(names)) if i != e]
    singles = []
    for a in non_e:
        for p in bld.conserving_products((a,)):
            singles.append((a, p))
    ionis = [(a, p) for a, p in singles if bld.charge[a] == 0 and e in p]
    others = [(a, p) for a, p in singles if not (bld.charge[a] == 0 and e in p)]
    chosen = list(ionis)
    if len(chosen) < n_cr:
        pick = rng.choice(len(others), size=n_cr - len(chosen), replace=False)
        chosen += [others[i] for i in sorted(pick)]
    for a, p in chosen[:n_cr]:
        bld.add(COSMIC_RAY, (a,), p, _loguniform(rng, 0.1, 10.0), 0.0, 0.0)
    # two-body reactions grown from the atomic start: the initial atoms and
    # whatever the cosmic-ray set makes from reachable species
    reach = np.zeros(len(names), bool)
    reach[[names.index(a) for a in ("H", "C", "O")]] = True
    changed = True
    while changed:
        changed = False
        for t_, rs, ps, *_ in bld.rows:
            if all(reach[r] for r in rs) and not all(reach[p] for p in ps):
                reach[list(ps)] = True
                changed = True
    ion_neutral = lambda a, b: a != e and b != e and not (bld.charge[a] != 0 and bld.charge[b] != 0)
    bld.grow(reach, [TWO_BODY] * n_two_body, ion_neutral, None, e)
    return bld.build()


# ---------------------------------------------------------------------------
# large {H, He, C, N, O, S} networks
# ---------------------------------------------------------------------------
MANDATORY = [
    (_comp(), -1),
    (_comp(H=1), 0), (_comp(H=1), 1), (_comp(H=2), 0), (_comp(H=2), 1), (_comp(H=3), 1),
    (_comp(He=1), 0), (_comp(He=1), 1),
    (_comp(C=1), 0), (_comp(C=1), 1), (_comp(N=1), 0), (_comp(N=1), 1),
    (_comp(O=1), 0), (_comp(O=1), 1), (_comp(S=1), 0), (_comp(S=1), 1),
    (_comp(C=1, O=1), 0), (_comp(H=1, C=1, O=1), 1),
]


def _candidate_species():
    out = []
    for a in range(0, 7):
        for b, c, d, e in itertools.product(range(5), repeat=4):
            if b + c + d + e > 4 or a + b + c + d + e == 0:
                continue
            comp = (a, 0, b, c, d, e)
            out.append((comp, 0))
            out.append((comp, 1))
    return out


def large_network(n_species: int, n_reactions: int, seed: int,
                  mix=(0.8, 0.1, 0.1)) -> Network:
    """n_species over {H, He, C, N, O, S} + charge with the two-body / cosmic-ray /
    photo reaction mix `mix` (exact counts, two-body takes the rounding rest)."""
    rng = np.random.default_rng(seed)
    mandatory = list(MANDATORY)
    cand = [c for c in _candidate_species() if c not in mandatory]
    if n_species < len(mandatory) or n_species > len(mandatory) + len(cand):
        raise ValueError("n_species out of range")
    pick = rng.choice(len(cand), size=n_species - len(mandatory), replace=False)
    chosen = mandatory + [cand[i] for i in sorted(pick)]
    electron = chosen[0]
    rest = sorted(chosen[1:], key=lambda t: (sum(t[0]), t[0], t[1]))
    chosen = [electron] + rest
    names = [species_name(c, q) for c, q in chosen]
    comp = [c for c, _ in chosen]
    charge = [q for _, q in chosen]
    bld = _Builder(f"large-{n_species}-{n_reactions}-{seed}", names, comp, charge, rng)
    e = 0
    n_cr = int(round(mix[1] * n_reactions))
    n_ph = int(round(mix[2] * n_reactions))
    n_2b = n_reactions - n_cr - n_ph
    # neutral-neutral, neutral-cation and electron-cation pairs; no ion-ion pair
    q = bld.charge

    def allowed(a, b):
        if a == e:
            return b != e and q[b] > 0
        return (q[a] == 0 and q[b] >= 0) or (q[a] > 0 and q[b] == 0)

    def single_ok(kind, a):
        return a != e
    # reactions grown from the atomic start, types in a seeded order with exact counts
    kinds = np.array([TWO_BODY] * n_2b + [COSMIC_RAY] * n_cr + [PHOTO] * n_ph)
    kinds = kinds[rng.permutation(len(kinds))]
    # the first reactions ionise: the atoms alone allow neutral-neutral and
    # cosmic-ray chemistry, the rest follows from what they make
    reach = np.zeros(n_species, bool)
    for atom in ("H", "He", "C", "N", "O", "S"):
        reach[names.index(atom)] = True
    bld.grow(reach, list(kinds), allowed, single_ok, e)
    return bld.build()


_CONFIG_NETS = {
    "small": lambda: small_network(seed=1),
    "net200": lambda: large_network(200, 2500, seed=200),
    "net500": lambda: large_network(500, 6000, seed=500),
}
_CACHE: dict = {}


def network_for_config(name: str) -> Network:
    """The fixed seeded networks: 'small' (12/40), 'net200' (200/2500), 'net500' (500/6000)."""
    if name not in _CACHE:
        _CACHE[name] = _CONFIG_NETS[name]()
    return _CACHE[name]


def make_network(name, species, reactions, albedo=0.0) -> Network:
    """Explicit network.  species: [(name, {element: count}, charge)];
    reactions: [(rtype, [reactant names], [product names], alpha, beta, gamma)].
    Raises ValueError if a reaction does not conserve every element and charge."""
    names = [s[0] for s in species]
    comp = np.array([_comp(**s[1]) for s in species], dtype=np.int64)
    charge = np.array([s[2] for s in species], dtype=np.int64)
    R = len(reactions)
    rtype = np.zeros(R, np.int32)
    rea = -np.ones((R, 2), np.int32)
    pro = -np.ones((R, 3), np.int32)
    al, be, ga = np.zeros(R), np.zeros(R), np.zeros(R)
    for r, (t, rs, ps, a, b, g) in enumerate(reactions):
        ri = sorted(names.index(s) for s in rs)
        pi = sorted(names.index(s) for s in ps)
        if not (1 <= len(ri) <= 2 and 1 <= len(pi) <= 3):
            raise ValueError(f"reaction {r}: 1-2 reactants and 1-3 products required")
        if (comp[ri].sum(0) != comp[pi].sum(0)).any() or charge[ri].sum() != charge[pi].sum():
            raise ValueError(f"reaction {r} does not conserve elements and charge")
        rtype[r] = t
        rea[r, : len(ri)] = ri
        pro[r, : len(pi)] = pi
        al[r], be[r], ga[r] = a, b, g
    return Network(name, names, comp, charge, rtype, rea, pro, al, be, ga, albedo)
