"""Stencil-program texts used as inputs by the language tests (the same text
goes to the interpreter and to the compiled kernel)."""

import numpy as np

from paper_2310_01882_amd.programs import JACOBI, advection  # noqa: F401


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
