"""CPU: consistency checks on the kernel sources that the compiler cannot make.

The batch kernels read each member's argument record field by field (load_unit); a field
added to KArgs or Geom but not copied there would reach the kernels uninitialised."""
import os
import re

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2404_13683_amd", "csrc", "kernels.hpp")


def _struct_fields(text, name):
    body = re.search(r"struct %s \{(.*?)\n\};" % name, text, re.S).group(1)
    body = re.sub(r"//[^\n]*", "", body)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split()[-1] if "," not in decl else decl
        for part in names.split(","):
            fields.append(part.strip().split()[-1].lstrip("*"))
    return fields


def test_load_unit_copies_every_field():
    text = open(SRC).read()
    geom = _struct_fields(text, "Geom")
    kargs = _struct_fields(text, "KArgs")
    assert "g" in kargs and "u" in kargs and "unit_tr" in kargs and "nx" in geom
    body = re.search(r"KArgs load_unit\(.*?\n\}", text, re.S).group(0)
    copied = set(re.findall(r"a\.([a-z_0-9.]+) = p->\1;", body))
    expected = {"g." + f for f in geom} | {f for f in kargs if f != "g"}
    assert copied == expected, (sorted(expected - copied), sorted(copied - expected))
