"""Model files in the plain-text format of the paper's model parser (section 5,
"Model parser" table): one file gives the initial state, the reactions with
their rate constants, the final time and the number of output points.

    // simple model of a predator-prey oscillation
    # init
    A = 1000
    B = 1000
    # reactions
    1 A --> 2 A : 10
    1 A 1 B --> 2 B : 0.01
    1 B --> NULL : 10
    # end
    time = 2
    steps = 10000

* ``//`` starts a comment (whole line or trailing); blank lines are ignored.
* ``# init``: ``<species> = <count>``; the order of these lines fixes the
  species index.
* ``# reactions``: ``<coef> <species> [<coef> <species> ...] --> <coef>
  <species> ... : <rate>``; ``NULL`` stands for an empty side.  A species
  named twice on one side has its coefficients added.  Reactants may total
  at most 2 molecules (mass action as in Eq. 1-2; the paper rewrites higher
  orders as steps of order <= 2).
* ``# end``, then ``time = <t_end>`` and ``steps = <number of output
  points>``; the output points are evenly spaced on [0, t_end], both ends
  included.

This module only reads and writes text and builds input arrays (through
``workloads.from_reactions``); it holds none of the simulation's arithmetic.
"""
from __future__ import annotations

import math
import re
from typing import NamedTuple

import numpy as np

from . import workloads as W

__all__ = ["Model", "parse", "load", "dumps", "save", "sample_grid"]


class Model(NamedTuple):
    net: W.NetSpec          # species names are net.names
    x0: np.ndarray          # int32 [N]
    t_end: float
    steps: int              # number of output points


class ModelFileError(ValueError):
    pass


_NAME = re.compile(r"[A-Za-z_][A-Za-z0-9_.\-']*$")


def _fail(lineno: int, msg: str):
    raise ModelFileError("line %d: %s" % (lineno, msg))


def _side(text: str, species: dict, lineno: int) -> dict:
    toks = text.split()
    if toks == ["NULL"] or not toks:
        if not toks:
            _fail(lineno, "empty reaction side (write NULL)")
        return {}
    if len(toks) % 2:
        _fail(lineno, "a side must be pairs '<coef> <species>' or NULL")
    out: dict = {}
    for i in range(0, len(toks), 2):
        c, name = toks[i], toks[i + 1]
        if not c.isdigit() or int(c) < 1:
            _fail(lineno, "coefficient %r is not a positive integer" % c)
        if name == "NULL":
            _fail(lineno, "NULL cannot be combined with species")
        if name not in species:
            _fail(lineno, "species %r is not declared in # init" % name)
        j = species[name]
        out[j] = out.get(j, 0) + int(c)
    return out


def parse(text: str) -> Model:
    """Parse a model file's text into a Model."""
    section = None
    names: list = []
    index: dict = {}
    counts: list = []
    reactions: list = []
    settings: dict = {}
    seen = set()
    for lineno, raw in enumerate(text.splitlines(), 1):
        line = raw.split("//", 1)[0].strip()
        if not line:
            continue
        if line.startswith("#"):
            tag = line[1:].strip().lower()
            if tag not in ("init", "reactions", "end"):
                _fail(lineno, "unknown section %r" % line)
            if tag in seen:
                _fail(lineno, "section %r given twice" % line)
            order = ["init", "reactions", "end"]
            if [t for t in order if t in seen] != order[:len(seen)] or order[len(seen)] != tag:
                _fail(lineno, "sections must come in the order # init, # reactions, # end")
            seen.add(tag)
            section = tag
            continue
        if section is None:
            _fail(lineno, "text before '# init'")
        if section == "init":
            if "=" not in line:
                _fail(lineno, "expected '<species> = <count>'")
            name, val = (s.strip() for s in line.split("=", 1))
            if not _NAME.match(name) or name == "NULL":
                _fail(lineno, "bad species name %r" % name)
            if name in index:
                _fail(lineno, "species %r declared twice" % name)
            if not val.isdigit() or int(val) > 2**31 - 1:
                _fail(lineno, "count %r is not an integer in [0, 2^31 - 1]" % val)
            index[name] = len(names)
            names.append(name)
            counts.append(int(val))
        elif section == "reactions":
            if "-->" not in line or ":" not in line:
                _fail(lineno, "expected '<reactants> --> <products> : <rate>'")
            lhs, rest = line.split("-->", 1)
            rhs, rate = rest.rsplit(":", 1)
            try:
                c = float(rate)
            except ValueError:
                _fail(lineno, "rate %r is not a number" % rate.strip())
            if not (math.isfinite(c) and c >= 0.0):
                _fail(lineno, "rate must be finite and >= 0")
            reac = _side(lhs, index, lineno)
            prod = _side(rhs, index, lineno)
            if sum(reac.values()) > 2:
                _fail(lineno, "more than 2 reactant molecules; rewrite it as steps of order <= 2")
            reactions.append((reac, prod, c))
        else:
            if "=" not in line:
                _fail(lineno, "expected 'time = <t_end>' or 'steps = <points>'")
            key, val = (s.strip() for s in line.split("=", 1))
            if key not in ("time", "steps"):
                _fail(lineno, "unknown setting %r" % key)
            if key in settings:
                _fail(lineno, "setting %r given twice" % key)
            settings[key] = (val, lineno)
    if seen != {"init", "reactions", "end"}:
        raise ModelFileError("missing section(s): %s" % ", ".join(
            "# " + t for t in ("init", "reactions", "end") if t not in seen))
    if not names:
        raise ModelFileError("no species in # init")
    if not reactions:
        raise ModelFileError("no reactions in # reactions")
    for key in ("time", "steps"):
        if key not in settings:
            raise ModelFileError("missing setting %r after # end" % key)
    tval, tl = settings["time"]
    try:
        t_end = float(tval)
    except ValueError:
        _fail(tl, "time %r is not a number" % tval)
    if not (math.isfinite(t_end) and t_end >= 0.0):
        _fail(tl, "time must be finite and >= 0")
    sval, sl = settings["steps"]
    if not sval.isdigit() or int(sval) < 1:
        _fail(sl, "steps %r is not a positive integer" % sval)
    net = W.from_reactions(len(names), reactions, names=names)
    return Model(net, np.asarray(counts, dtype=np.int32), t_end, int(sval))


def load(path: str) -> Model:
    with open(path) as f:
        return parse(f.read())


def _fmt_side(entries) -> str:
    return " ".join("%d %s" % (m, s) for s, m in entries) if entries else "NULL"


def dumps(model: Model, comment: str = "") -> str:
    """Model file text for a Model; parse(dumps(m)) rebuilds m exactly."""
    net = model.net
    names = list(net.names) if net.names else ["S%d" % j for j in range(net.N)]
    if len(names) != net.N or len(set(names)) != net.N:
        raise ModelFileError("species names must be N distinct names")
    lines = ["// " + c for c in comment.splitlines()] if comment else []
    lines.append("# init")
    for j in range(net.N):
        lines.append("%s = %d" % (names[j], int(model.x0[j])))
    lines.append("# reactions")
    for k in range(net.M):
        reac = [(names[net.react_species[e]], int(net.react_sigma[e]))
                for e in range(net.react_ptr[k], net.react_ptr[k + 1])]
        prod = [(names[net.prod_species[e]], int(net.prod_mult[e]))
                for e in range(net.prod_ptr[k], net.prod_ptr[k + 1])]
        lines.append("%s --> %s : %s" % (_fmt_side(reac), _fmt_side(prod), repr(float(net.c[k]))))
    lines.append("# end")
    lines.append("time = %s" % repr(float(model.t_end)))
    lines.append("steps = %d" % int(model.steps))
    return "\n".join(lines) + "\n"


def save(model: Model, path: str, comment: str = ""):
    with open(path, "w") as f:
        f.write(dumps(model, comment))


def sample_grid(model: Model) -> np.ndarray:
    """The model's output points: `steps` points evenly spaced on [0, t_end]."""
    return W.uniform_grid(model.t_end, model.steps)
