"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and rejects bad model descriptions before touching a device."""
import os
import re

import pytest

from paper_2505_12414_amd import uml, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "uml.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(uml_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 20
    L = uml.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(uml.SIGNATURES), "binding and header disagree"


def test_version_and_error_plumbing():
    assert uml.uml_version() == "0.1.0"


def bad(desc_mod):
    d = W.mass1d()
    desc_mod(d)
    return d


@pytest.mark.parametrize("mod,code", [
    (lambda d: d["nodes"][0].update(params=[0]), uml.UML_E_INVALID),          # Gauss needs 2
    (lambda d: d["nodes"][1].update(dims=[3]), uml.UML_E_INVALID),            # bad dim index
    (lambda d: d["nodes"][2].update(children=[0, 2]), uml.UML_E_INVALID),     # self child
    (lambda d: d.update(root=7), uml.UML_E_INVALID),
    (lambda d: d["dims"][0].update(lo=6.0), uml.UML_E_INVALID),               # lo > hi
    (lambda d: d["nodes"].__setitem__(2, {"kind": "prod", "children": [0, 1]}),
     uml.UML_E_INVALID),                                                      # m used twice
])
def test_invalid_descriptions_are_rejected(mod, code):
    with pytest.raises(uml.UmlError) as e:
        uml.Model(bad(mod))
    assert e.value.code == code


def test_pwave_needs_its_ranges():
    d = W.pwave3d()
    d["dims"][2]["hi"] = 3.0
    with pytest.raises(uml.UmlError) as e:
        uml.Model(d)
    assert e.value.code == uml.UML_E_INVALID and "P-wave" in str(e.value)
