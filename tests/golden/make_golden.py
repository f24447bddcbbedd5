"""Writes tests/golden/quad_n1.txt from the closed form of the one-term
relative-error minimax fit of 1/y on [1, R] (equioscillation at y = 1,
y = 1/alpha and y = R).  Calls no product code."""
import math
import os

rows = []
for R in (10.0, 133.0, 1242.0, 14500.0):
    al = math.log(R) / (R - 1.0)
    be = 2.0 / (math.exp(-al) + 1.0 / (al * math.e))
    rows.append(f"{R:.6g} {al:.17g} {be:.17g} {1.0 - be * math.exp(-al):.17g}")
path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "quad_n1.txt")
with open(path, "w") as f:
    f.write("# R alpha beta E : one-term minimax exponential fit of 1/y on [1, R]\n")
    f.write("\n".join(rows) + "\n")
