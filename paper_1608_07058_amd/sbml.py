"""SBML-lite import: a mass-action subset of SBML into the flat network table.

The paper's models are SBML files loaded through libSBML (Implementation
section): species with initial amounts, reactions with reactant and product
stoichiometry, and kinetic laws.  This reader takes the subset the simulation
method needs -- mass-action reactions -- and returns a
``workloads.Network`` (reactant orders m[j][i], product coefficients
p[j][i], rate constants theta_j, initial copy numbers x0), which
``lx.Network(net.m, net.p)`` compiles.  It runs on the host and uses only the
standard library's XML parser.

Accepted (SBML Level 2 or 3, any namespace):
  * species with ``initialAmount`` (a copy number), or ``initialConcentration``
    times the size of its compartment; ``boundaryCondition="true"`` or
    ``constant="true"`` species are held fixed: they are dropped from the
    table and their amount is folded into the rate constants of the
    reactions that read them;
  * reactions whose kinetic law (MathML) is a mass-action term
    ``k * S1 * S2 ...`` -- a product of one parameter (local, or global from
    listOfParameters; numbers multiply in as well) and the reactant species,
    each appearing as many times as its stoichiometry (``<power>`` with an
    integer exponent is accepted too), optionally times compartment sizes;
  * reversible reactions whose law is the difference of two such terms,
    ``k_f * reactants - k_b * products``: they become two reactions, forward
    then backward.

Reading of the rate constant: the kinetic law k * prod_i S_i^{m_i} is the
large-copy-number form of the propensity, so the stochastic constant of the
combinatorial propensity theta * prod_i C(x_i, m_i) is
theta = k * prod_i m_i! (e.g. 2A -> B with law k*A*A gives theta = 2k).
Compartment sizes in the law multiply into k.  Anything else (rules,
events, function definitions, non-mass-action laws, non-integer
stoichiometry, reaction order above 3) is rejected with SbmlError naming the
element.
"""

from __future__ import annotations

import math
import xml.etree.ElementTree as ET

import numpy as np

from . import workloads

class SbmlError(ValueError):
    """The document is outside the mass-action subset this reader accepts."""


def _local(tag: str) -> str:
    return tag.rsplit("}", 1)[-1]


def _children(el, name):
    return [c for c in el if _local(c.tag) == name]


def _child(el, name):
    out = _children(el, name)
    return out[0] if out else None


def _items(el, list_name, *item_names):
    """The items of the list element `list_name` under `el` (none if absent)."""
    lst = _child(el, list_name)
    if lst is None:
        return []
    return [c for c in lst if _local(c.tag) in item_names]


def _float(el, attr, what):
    v = el.get(attr)
    if v is None:
        raise SbmlError(f"{what}: missing attribute {attr!r}")
    try:
        return float(v)
    except ValueError:
        raise SbmlError(f"{what}: attribute {attr!r} is not a number: {v!r}") from None


class _Term:
    """A product coefficient * prod(symbol ^ power) from MathML."""

    def __init__(self):
        self.coef = 1.0
        self.syms = {}  # name -> power

    def mul_sym(self, name, power=1):
        self.syms[name] = self.syms.get(name, 0) + power


def _term(node, what):
    """Parse a MathML product (apply/times, ci, cn, apply/power) into a _Term."""
    t = _Term()

    def walk(n):
        tag = _local(n.tag)
        if tag == "ci":
            t.mul_sym(n.text.strip())
        elif tag == "cn":
            t.coef *= float(n.text.strip())
        elif tag == "apply":
            op = _local(n[0].tag)
            args = list(n)[1:]
            if op == "times":
                for a in args:
                    walk(a)
            elif op == "power":
                if len(args) != 2 or _local(args[0].tag) != "ci" or _local(args[1].tag) != "cn":
                    raise SbmlError(f"{what}: only species ^ integer powers are accepted")
                e = float(args[1].text.strip())
                if e != int(e) or e < 1:
                    raise SbmlError(f"{what}: non-integer power {e}")
                t.mul_sym(args[0].text.strip(), int(e))
            else:
                raise SbmlError(f"{what}: the kinetic law is not a mass-action product "
                                f"(operator {op!r})")
        else:
            raise SbmlError(f"{what}: unexpected MathML element {tag!r}")

    walk(node)
    return t


def _law_terms(kl, what):
    """The kinetic law as one term (irreversible) or two (forward - backward)."""
    math_el = _child(kl, "math")
    if math_el is None or len(math_el) != 1:
        raise SbmlError(f"{what}: kinetic law without a single MathML expression")
    top = math_el[0]
    if _local(top.tag) == "apply" and _local(top[0].tag) == "minus":
        args = list(top)[1:]
        if len(args) != 2:
            raise SbmlError(f"{what}: unary minus in a kinetic law")
        return [_term(args[0], what), _term(args[1], what)]
    return [_term(top, what)]


def _stoich(ref, what):
    s = ref.get("stoichiometry", "1")
    try:
        v = float(s)
    except ValueError:
        raise SbmlError(f"{what}: stoichiometry {s!r} is not a number") from None
    if v != int(v) or v < 0:
        raise SbmlError(f"{what}: stoichiometry must be a non-negative integer, got {s}")
    if _child(ref, "stoichiometryMath") is not None:
        raise SbmlError(f"{what}: stoichiometryMath is not supported")
    return int(v)


def read_sbml(source) -> workloads.Network:
    """Read an SBML document (path, file object or XML string) into a Network.

    Returns a ``workloads.Network`` whose species are the non-fixed species
    in document order and whose reactions are the document's reactions in
    order (a reversible one as forward, backward)."""
    if hasattr(source, "read"):
        root = ET.parse(source).getroot()
    elif isinstance(source, str) and source.lstrip().startswith("<"):
        root = ET.fromstring(source)
    else:
        root = ET.parse(source).getroot()
    if _local(root.tag) != "sbml":
        raise SbmlError("not an SBML document")
    model = _child(root, "model")
    if model is None:
        raise SbmlError("no model element")
    for bad in ("listOfRules", "listOfEvents", "listOfFunctionDefinitions",
                "listOfInitialAssignments", "listOfConstraints"):
        lst = _child(model, bad)
        if lst is not None and len(lst):
            raise SbmlError(f"{bad} is not supported by the mass-action subset")

    sizes = {}
    for c in _items(model, "listOfCompartments", "compartment"):
        sizes[c.get("id")] = float(c.get("size", c.get("volume", "1")))
    params = {}
    for p in _items(model, "listOfParameters", "parameter"):
        params[p.get("id")] = _float(p, "value", f"parameter {p.get('id')}")

    species, fixed, amount = [], {}, {}
    for s in _items(model, "listOfSpecies", "species"):
        sid = s.get("id")
        what = f"species {sid}"
        if s.get("initialAmount") is not None:
            a = _float(s, "initialAmount", what)
        elif s.get("initialConcentration") is not None:
            a = _float(s, "initialConcentration", what) * sizes.get(s.get("compartment"), 1.0)
        else:
            raise SbmlError(f"{what}: no initial amount")
        if a < 0 or a != round(a):
            raise SbmlError(f"{what}: initial amount {a} is not a copy number")
        if s.get("boundaryCondition") == "true" or s.get("constant") == "true":
            fixed[sid] = a
        else:
            species.append(sid)
            amount[sid] = int(round(a))
    index = {sid: i for i, sid in enumerate(species)}
    N = len(species)
    if N == 0:
        raise SbmlError("no species")

    rows_m, rows_p, theta, names = [], [], [], []
    for r in _items(model, "listOfReactions", "reaction"):
        rid = r.get("id")
        what = f"reaction {rid}"
        side = {}
        for lst, key in (("listOfReactants", "m"), ("listOfProducts", "p")):
            vec = np.zeros(N, np.int32)
            fixed_in = {}
            for ref in _items(r, lst, "speciesReference"):
                sp = ref.get("species")
                k = _stoich(ref, what)
                if sp in index:
                    vec[index[sp]] += k
                elif sp in fixed:
                    fixed_in[sp] = fixed_in.get(sp, 0) + k
                else:
                    raise SbmlError(f"{what}: unknown species {sp!r}")
            side[key] = (vec, fixed_in)
        if _items(r, "listOfModifiers", "modifierSpeciesReference"):
            raise SbmlError(f"{what}: modifiers are outside the mass-action subset")
        kl = _child(r, "kineticLaw")
        if kl is None:
            raise SbmlError(f"{what}: no kinetic law")
        local = dict(params)
        for lst in ("listOfParameters", "listOfLocalParameters"):
            for p in _items(kl, lst, "parameter", "localParameter"):
                local[p.get("id")] = _float(p, "value", f"{what}: parameter {p.get('id')}")
        terms = _law_terms(kl, what)
        # a single mass-action term is one irreversible reaction (SBML Level 2
        # defaults `reversible` to true, so the attribute alone decides nothing);
        # a difference of two terms is a reversible pair
        if len(terms) == 2 and r.get("reversible") == "false":
            raise SbmlError(f"{what}: a difference law on an irreversible reaction")
        (rm, rm_fixed), (rp, rp_fixed) = side["m"], side["p"]
        dirs = [(rm, rm_fixed, rp, terms[0])]
        if len(terms) == 2:
            dirs.append((rp, rp_fixed, rm, terms[1]))
        for q, (reac, reac_fixed, prod, term) in enumerate(dirs):
            k = term.coef
            want = {species[i]: int(reac[i]) for i in range(N) if reac[i]}
            want.update(reac_fixed)
            got = {}
            for name, pw in term.syms.items():
                if name in index or name in fixed:
                    got[name] = pw
                elif name in sizes:
                    k *= sizes[name] ** pw
                elif name in local:
                    k *= local[name] ** pw
                else:
                    raise SbmlError(f"{what}: unknown symbol {name!r} in the kinetic law")
            if got != want:
                raise SbmlError(f"{what}: the kinetic law is not mass action in its reactants "
                                f"(law has {got}, reactants are {want})")
            order = int(reac.sum()) + sum(reac_fixed.values())
            if order > 3:
                raise SbmlError(f"{what}: reaction order {order} above 3")
            # stochastic constant of the combinatorial propensity; the amounts of
            # fixed species fold into it
            for i in range(N):
                k *= math.factorial(int(reac[i]))
            for sp, mult in reac_fixed.items():
                k *= fixed[sp] ** mult
            if not (k >= 0.0) or math.isinf(k):
                raise SbmlError(f"{what}: rate constant {k} is not a finite non-negative number")
            rows_m.append(reac.copy())
            rows_p.append(prod.copy())
            theta.append(k)
            names.append(rid if len(dirs) == 1 else rid + ("_fwd" if q == 0 else "_bwd"))
    if not rows_m:
        raise SbmlError("no reactions")
    model_id = model.get("id") or model.get("name") or "sbml"
    return workloads._net(model_id, np.array(rows_m), np.array(rows_p), theta,
                          [amount[s] for s in species], tuple(species), tuple(names))
