"""The evaluation's two benchmarks written in the stencil-program language
(Section 4.1): the 7-point Jacobi update of the Poisson problem and the
three-field advection source term on the staggered C-grid, as one region
with three outputs. Each operation appears in the order the hand-written
kernels evaluate it, so a compiled program reproduces them bit for bit."""

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
    outputs (staggered C-grid: u at i+1/2, v at j+1/2, w at k+1/2; per
    field, x, y and z flux differences weighted by tcx, tcy and the
    per-level tzc1 / tzc2)."""
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

ADVECTION = advection()
