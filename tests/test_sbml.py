"""SBML-lite import (mass-action subset) into the flat network table, on
SBML documents written by hand (tests/golden/*.xml)."""

import os

import numpy as np
import pytest

from paper_1608_07058_amd import sbml, workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_dimer_level3_matches_the_table():
    net = sbml.read_sbml(os.path.join(GOLDEN, "dimer_l3.xml"))
    ref = W.dimer()
    assert net.species == ("S1", "S2", "S3")
    assert net.reactions == ("decay", "dimerize_fwd", "dimerize_bwd", "convert")
    assert np.array_equal(net.m, ref.m) and np.array_equal(net.p, ref.p)
    # 2 S1 -> S2 with law k2 S1^2: theta = 2! k2 = 0.002
    assert np.allclose(net.theta, ref.theta, rtol=1e-15)
    assert np.array_equal(net.x0, ref.x0)


def test_birth_death_level2_fixed_species_and_volume():
    net = sbml.read_sbml(os.path.join(GOLDEN, "birth_death_l2.xml"))
    ref = W.birth_death()
    assert net.species == ("X",)
    assert np.array_equal(net.m, ref.m) and np.array_equal(net.p, ref.p)
    # source amount 2 folds into k1 = 5; the volume 0.5 into kd = 0.2
    assert np.allclose(net.theta, ref.theta, rtol=1e-15)
    assert net.x0.tolist() == [0]


def test_imported_table_compiles_in_the_oracle(orc):
    net = sbml.read_sbml(os.path.join(GOLDEN, "dimer_l3.xml"))
    th, x0 = W.tile(net, 8)
    res = orc.simulate(net.m, net.p, th, x0, 1.0)
    ref = orc.simulate(W.dimer().m, W.dimer().p, th, x0, 1.0)
    for k in ("x", "r", "G"):
        assert np.array_equal(res[k], ref[k])


def _doc(reactions, species='<species id="A" compartment="c" initialAmount="10"/>', extra=""):
    return f"""<sbml xmlns="http://www.sbml.org/sbml/level3/version1/core" level="3" version="1">
  <model id="t"><listOfCompartments><compartment id="c" size="1"/></listOfCompartments>
  <listOfSpecies>{species}<species id="B" compartment="c" initialAmount="0"/></listOfSpecies>
  {extra}<listOfReactions>{reactions}</listOfReactions></model></sbml>"""


def _law(mathml):
    return f'<kineticLaw><math xmlns="http://www.w3.org/1998/Math/MathML">{mathml}</math></kineticLaw>'


RX = '<listOfReactants><speciesReference species="A"/></listOfReactants>' \
     '<listOfProducts><speciesReference species="B"/></listOfProducts>'


@pytest.mark.parametrize("what,doc", [
    ("non-mass-action law", _doc(f'<reaction id="r">{RX}' + _law(
        "<apply><divide/><ci>A</ci><cn>2</cn></apply>") + "</reaction>")),
    ("law missing a reactant", _doc(f'<reaction id="r">{RX}' + _law("<cn>3</cn>") + "</reaction>")),
    ("unknown symbol", _doc(f'<reaction id="r">{RX}' + _law(
        "<apply><times/><ci>kk</ci><ci>A</ci></apply>") + "</reaction>")),
    ("non-integer stoichiometry", _doc(
        '<reaction id="r"><listOfReactants><speciesReference species="A" stoichiometry="1.5"/>'
        '</listOfReactants>' + _law("<apply><times/><cn>1</cn><ci>A</ci></apply>") + "</reaction>")),
    ("order above 3", _doc(
        '<reaction id="r"><listOfReactants><speciesReference species="A" stoichiometry="4"/>'
        '</listOfReactants>' + _law("<apply><times/><cn>1</cn><apply><power/><ci>A</ci><cn>4</cn>"
                                    "</apply></apply>") + "</reaction>")),
    ("rules", _doc("", extra='<listOfRules><assignmentRule variable="B"/></listOfRules>')),
    ("modifier", _doc(f'<reaction id="r">{RX}<listOfModifiers><modifierSpeciesReference '
                      f'species="B"/></listOfModifiers>' + _law(
                          "<apply><times/><cn>1</cn><ci>A</ci></apply>") + "</reaction>")),
    ("fractional amount", _doc(f'<reaction id="r">{RX}' + _law(
        "<apply><times/><cn>1</cn><ci>A</ci></apply>") + "</reaction>",
        species='<species id="A" compartment="c" initialAmount="2.5"/>')),
])
def test_outside_the_subset_is_rejected(what, doc):
    with pytest.raises(sbml.SbmlError):
        sbml.read_sbml(doc)


def test_reversible_law_and_power_forms():
    doc = _doc(f'<reaction id="r" reversible="true">{RX}' + _law(
        "<apply><minus/><apply><times/><cn>3</cn><ci>A</ci></apply>"
        "<apply><times/><cn>0.5</cn><ci>B</ci></apply></apply>") + "</reaction>")
    net = sbml.read_sbml(doc)
    assert net.m.tolist() == [[1, 0], [0, 1]] and net.p.tolist() == [[0, 1], [1, 0]]
    assert net.theta.tolist() == [3.0, 0.5]
    assert net.reactions == ("r_fwd", "r_bwd")
