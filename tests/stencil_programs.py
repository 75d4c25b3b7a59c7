"""Stencil-program texts used as inputs by the language tests (the same text
goes to the interpreter and to the compiled kernel)."""

import numpy as np

JACOBI = """
# one 7-point Jacobi update of the Poisson problem
field u, f;
let s = ((((u[1,0,0] + u[-1,0,0]) + u[0,1,0]) + u[0,-1,0]) + u[0,0,1]) + u[0,0,-1];
out v = (s - f) * 0.16666666666666666;
"""


def _flux(phi, side, vel, a, b):
    # phi at the neighbour on `side` times the sum of two velocity samples
    return f"({phi}[{side}] * ({vel}[{a}] + {vel}[{b}]))"


def advection() -> str:
    """The three-field advection source term as one region with three
    outputs (the staggered C-grid form of the advection row)."""
    rows = {
        "su": [("u", "-1,0,0", "u", "-1,0,0", "0,0,0"), ("u", "1,0,0", "u", "0,0,0", "1,0,0"),
               ("u", "0,-1,0", "v", "0,-1,0", "1,-1,0"), ("u", "0,1,0", "v", "0,0,0", "1,0,0"),
               ("u", "0,0,-1", "w", "0,0,-1", "1,0,-1"), ("u", "0,0,1", "w", "0,0,0", "1,0,0")],
        "sv": [("v", "-1,0,0", "u", "-1,0,0", "-1,1,0"), ("v", "1,0,0", "u", "0,0,0", "0,1,0"),
               ("v", "0,-1,0", "v", "0,-1,0", "0,0,0"), ("v", "0,1,0", "v", "0,0,0", "0,1,0"),
               ("v", "0,0,-1", "w", "0,0,-1", "0,1,-1"), ("v", "0,0,1", "w", "0,0,0", "0,1,0")],
        "sw": [("w", "-1,0,0", "u", "-1,0,0", "-1,0,1"), ("w", "1,0,0", "u", "0,0,0", "0,0,1"),
               ("w", "0,-1,0", "v", "0,-1,0", "0,-1,1"), ("w", "0,1,0", "v", "0,0,0", "0,0,1"),
               ("w", "0,0,-1", "w", "0,0,-1", "0,0,0"), ("w", "0,0,1", "w", "0,0,0", "0,0,1")],
    }
    text = "field u, v, w;\nparam tcx, tcy;\nprofile tzc1, tzc2;\n"
    for out, terms in rows.items():
        p = [_flux(*t) for t in terms]
        text += (f"out {out} = (tcx * ({p[0]} - {p[1]}) + tcy * ({p[2]} - {p[3]}))"
                 f" + (tzc1 * {p[4]} - tzc2 * {p[5]});\n")
    return text


def random_program(seed: int, depth: int = 4):
    """A random program over 3 fields, 2 params, 1 profile, 2 lets and 2
    outputs. Divisions are by (2 + x*x) so they stay finite."""
    g = np.random.Generator(np.random.PCG64(seed))

    def leaf(lets):
        r = g.integers(0, 5)
        if r == 0:
            return f"{g.uniform(-3, 3):.6g}"
        if r == 1:
            return ["p", "q"][g.integers(0, 2)]
        if r == 2:
            return "t"
        if r == 3 and lets:
            return lets[g.integers(0, len(lets))]
        o = g.integers(-1, 2, size=3)
        return f"{['a', 'b', 'c'][g.integers(0, 3)]}[{o[0]},{o[1]},{o[2]}]"

    def expr(d, lets):
        if d == 0 or g.random() < 0.2:
            return leaf(lets)
        op = g.integers(0, 6)
        x, y = expr(d - 1, lets), expr(d - 1, lets)
        if op == 0:
            return f"{x} + {y}"
        if op == 1:
            return f"{x} - ({y})"
        if op == 2:
            return f"({x}) * ({y})"
        if op == 3:
            return f"({x}) / (2 + ({y}) * ({y}))"
        if op == 4:
            return f"-({x})"
        return f"({x} - {y}) * {leaf(lets)}"

    text = "field a, b, c;\nparam p, q;\nprofile t;\n"
    lets = []
    for n in ("l0", "l1"):
        text += f"let {n} = {expr(depth, lets)};\n"
        lets.append(n)
    for n in ("o0", "o1"):
        text += f"out {n} = {expr(depth, lets)};\n"
    return text
