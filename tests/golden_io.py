"""Readers for the text fixtures under tests/golden/."""

import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                yield ln


def simplex(tok):
    """'3.2.1' -> (3, 2, 1)"""
    return tuple(int(v) for v in tok.split("."))


def rectangle():
    out = {"bars": []}
    for ln in lines("rectangle.txt"):
        key, _, rest = ln.partition(":")
        rest = rest.split()
        if key == "order":
            out["order"] = [simplex(t) for t in rest]
        elif key == "diam":
            out["diam"] = [float(t) for t in rest]
        elif key == "apparent":
            out["apparent"] = [tuple(simplex(s) for s in t.split(":")) for t in rest]
        elif key == "morse":
            out["morse"] = [int(t) for t in rest]
        elif key == "morse_printed":
            out["morse_printed"] = [int(t) for t in rest]
        elif key == "bar":
            d, b, de, bs, ds = rest
            out["bars"].append((int(d), float(b), float(de), simplex(bs),
                                None if ds == "-" else simplex(ds)))
    return out


def cns():
    vals, cof, fac = {}, None, None
    for ln in lines("cns.txt"):
        if ln.startswith("cofacets"):
            head, _, rest = ln.partition(":")
            cof = (simplex(head.split()[1]), int(head.split()[2][2:]), [int(t) for t in rest.split()])
        elif ln.startswith("facets"):
            head, _, rest = ln.partition(":")
            fac = (simplex(head.split()[1]), [int(t) for t in rest.split()])
        else:
            s, _, v = ln.partition("=")
            vals[simplex(s.strip())] = int(v)
    return vals, cof, fac


def column_counts():
    out = {}
    for ln in lines("column_counts.txt"):
        k, _, v = ln.partition("=")
        out[k.strip()] = int(v)
    return out
