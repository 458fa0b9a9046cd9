"""The C ABI header as documentation (CPU only): every entry point is preceded
by a comment, the five calls of the problem statement cite the passage of the
paper they implement, and the binding's structures have the header's layout."""
import ctypes as C
import os
import re

import pytest

from paper_2511_02257_amd import binding as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "cdag.h")
CORE = {"build_cdag": "Sec. II-B", "schedule": "Sec. III", "set_mem_budget": "Sec. II-C",
        "execute": "Sec. II-C", "fetch_correlators": "Sec. II-B"}


def declarations():
    """(name, comment) per function declared in the header, in order; the
    comment is the block right above the declaration, or above the group of
    declarations it belongs to (e.g. cdag_get_tile after cdag_set_tile)."""
    text = open(HEADER).read()
    token = re.compile(r"(?P<c>/\*.*?\*/)|(?P<d>^(?:int|const char\*)\s+(?P<n>\w+)\s*\([^;]*\);)|(?P<o>\S)",
                       re.S | re.M)
    out, comment = [], ""
    for m in token.finditer(text):
        if m.group("c"):
            comment = m.group("c")
        elif m.group("d"):
            out.append((m.group("n"), comment))
        else:
            comment = ""
    return out


def test_every_entry_point_has_a_comment():
    decls = declarations()
    assert len(decls) == len(B.EXPORTED)
    missing = [n for n, c in decls if len(c) < 20]
    assert not missing, missing


@pytest.mark.parametrize("name", sorted(CORE))
def test_core_calls_cite_their_passage(name):
    comment = dict(declarations())[name]
    assert comment.lstrip("/* ").startswith(name), comment[:80]
    assert CORE[name] in comment, (name, comment[:200])


def test_exec_stats_layout_matches_the_header():
    """Field names of cdag_exec_stats in the header, in order, equal the
    binding's structure (the sizes follow from the declared types)."""
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{\s*cdag_plan_stats plan;(.*?)\} cdag_exec_stats;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, rest = decl.split(None, 1)
        names += [x.strip() for x in rest.split(",")]
    assert ["plan"] + names == [n for n, _ in B.cdag_exec_stats._fields_]
    assert C.sizeof(B.cdag_exec_stats) == C.sizeof(B.cdag_plan_stats) + 8 * len(names)
