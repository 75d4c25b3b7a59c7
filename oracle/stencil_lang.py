"""Interpreter of the stencil-program language (a text form of a
stencil.apply region with an arbitrary arithmetic body).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.2 and Listing 2: a stencil.apply region reads its input temps at
constant offsets, combines the values with arith operations and yields the
output on the interior; Section 3 extracts such regions from Fortran loop
nests. The language states a region as declarations (field, param,
profile), named intermediate values (let) and outputs (out); expressions
have the usual precedence (unary minus, then * and /, then + and -), binary
operators group to the left, and every operation is one rounded operation
of the program's dtype, in the order the text gives.

The interpreter reads the text with its own tokenizer and recursive-descent
parser into nested tuples and evaluates them with numpy on whole interior
arrays.
"""

from __future__ import annotations

import re

import numpy as np

from .stencil import shifted

_NUM = re.compile(r"(\d+\.?\d*|\.\d+)([eE][+-]?\d+)?")
_NAME = re.compile(r"[A-Za-z_]\w*")
_KEYWORDS = {"field", "param", "profile", "let", "out"}
_LIMITS = {"field": 8, "param": 8, "profile": 4, "out": 4, "let": 256}


def _tokens(text: str):
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c.isspace():
            i += 1
            continue
        if c == "#":
            j = text.find("\n", i)
            i = n if j < 0 else j
            continue
        m = _NUM.match(text, i)
        if m:
            i = m.end()
            if i < n and (text[i].isalpha() or text[i] == "_"):
                raise ValueError("malformed number")
            out.append(("num", m.group()))
            continue
        m = _NAME.match(text, i)
        if m:
            out.append(("name", m.group()))
            i = m.end()
            continue
        out.append(("op", c))
        i += 1
    out.append(("end", ""))
    return out


class _Reader:
    def __init__(self, text):
        self.toks = _tokens(text)
        self.i = 0
        self.kinds = {}  # name -> kind
        self.decl = {"field": [], "param": [], "profile": [], "let": [], "out": []}
        self.lets = {}
        self.outs = []

    def peek(self):
        return self.toks[self.i]

    def take(self):
        t = self.toks[self.i]
        self.i += 1
        return t

    def want(self, op):
        t = self.take()
        if t != ("op", op):
            raise ValueError(f"expected '{op}'")

    def name(self):
        kind, text = self.take()
        if kind != "name":
            raise ValueError("expected a name")
        if text in _KEYWORDS:
            raise ValueError(f"'{text}' is a reserved word")
        return text

    def define(self, name, kind):
        if name in self.kinds:
            raise ValueError(f"'{name}' is already defined")
        self.kinds[name] = kind
        self.decl[kind].append(name)
        if len(self.decl[kind]) > _LIMITS[kind]:
            raise ValueError(f"too many {kind} declarations")

    def program(self):
        while self.peek()[0] != "end":
            kind, word = self.take()
            if kind != "name" or word not in _KEYWORDS:
                raise ValueError("expected a statement")
            if word in ("field", "param", "profile"):
                self.define(self.name(), word)
                while self.peek() == ("op", ","):
                    self.take()
                    self.define(self.name(), word)
            else:
                n = self.name()
                self.want("=")
                e = self.sum()
                self.define(n, word)
                if word == "let":
                    self.lets[n] = e
                else:
                    self.outs.append((n, e))
            self.want(";")
        if not self.outs:
            raise ValueError("the program has no output")

    # sum := product (('+'|'-') product)* ; grouped to the left
    def sum(self):
        e = self.product()
        while self.peek() in (("op", "+"), ("op", "-")):
            op = self.take()[1]
            e = (op, e, self.product())
        return e

    def product(self):
        e = self.signed()
        while self.peek() in (("op", "*"), ("op", "/")):
            op = self.take()[1]
            e = (op, e, self.signed())
        return e

    def signed(self):
        if self.peek() == ("op", "-"):
            self.take()
            return ("neg", self.signed())
        return self.atom()

    def offset(self):
        sign = 1
        if self.peek() == ("op", "-"):
            self.take()
            sign = -1
        kind, text = self.take()
        if kind != "num" or not text.isdigit():
            raise ValueError("expected an integer offset")
        v = sign * int(text)
        if not -1 <= v <= 1:
            raise ValueError("offsets must lie in [-1, 1]")
        return v

    def atom(self):
        kind, text = self.take()
        if (kind, text) == ("op", "("):
            e = self.sum()
            self.want(")")
            return e
        if kind == "num":
            v = float(text)
            if not np.isfinite(v):
                raise ValueError("constant out of range")
            return ("const", v)
        if kind != "name" or text not in self.kinds or self.kinds[text] == "out":
            raise ValueError(f"'{text}' is not defined")
        what = self.kinds[text]
        if self.peek() == ("op", "["):
            if what != "field":
                raise ValueError("only fields take offsets")
            self.take()
            dx = self.offset()
            self.want(",")
            dy = self.offset()
            self.want(",")
            dz = self.offset()
            self.want("]")
            return ("field", text, dx, dy, dz)
        if what == "field":
            return ("field", text, 0, 0, 0)
        return (what, text)


def parse(text: str) -> dict:
    """Parse a program; returns its declarations (names in order), lets and
    outputs as nested tuples. Raises ValueError on any error."""
    r = _Reader(text)
    r.program()
    return {"fields": r.decl["field"], "params": r.decl["param"],
            "profiles": r.decl["profile"], "lets": r.lets, "outputs": r.outs}


def run(text: str, fields, params=(), profiles=(), dtype=np.float64, interior_shape=None):
    """Evaluate a program on halo-padded (nz+2, ny+2, nx+2) fields; returns the
    interior arrays of the outputs in declaration order. ``fields``,
    ``params`` and ``profiles`` follow the declaration order; a program
    without fields needs ``interior_shape`` = (nz, ny, nx)."""
    prog = parse(text)
    dt = np.dtype(dtype).type
    if (len(fields) != len(prog["fields"]) or len(params) != len(prog["params"])
            or len(profiles) != len(prog["profiles"])):
        raise ValueError("argument counts differ from the declarations")
    arrays = {n: np.asarray(a, dtype=dtype) for n, a in zip(prog["fields"], fields)}
    if arrays:
        shape = next(iter(arrays.values())).shape
        interior_shape = (shape[0] - 2, shape[1] - 2, shape[2] - 2)
    elif interior_shape is None:
        raise ValueError("interior_shape is needed for a program without fields")
    nz = interior_shape[0]
    pvals = {n: dt(float(v)) for n, v in zip(prog["params"], params)}
    zvals = {n: np.asarray(t, dtype=dtype).reshape(nz, 1, 1)
             for n, t in zip(prog["profiles"], profiles)}
    letv = {}

    def ev(e):
        tag = e[0]
        if tag == "const":
            return dt(e[1])
        if tag == "field":
            return shifted(arrays[e[1]], e[2], e[3], e[4])
        if tag == "param":
            return pvals[e[1]]
        if tag == "profile":
            return zvals[e[1]]
        if tag == "let":
            return letv[e[1]]
        if tag == "neg":
            return np.negative(ev(e[1]))
        a, b = ev(e[1]), ev(e[2])
        if tag == "+":
            return a + b
        if tag == "-":
            return a - b
        if tag == "*":
            return a * b
        return a / b

    with np.errstate(all="ignore"):
        for name, e in prog["lets"].items():
            letv[name] = ev(e)
        outs = []
        for _, e in prog["outputs"]:
            v = np.broadcast_to(ev(e), tuple(interior_shape))
            outs.append(np.array(v, dtype=dtype))
    return outs
