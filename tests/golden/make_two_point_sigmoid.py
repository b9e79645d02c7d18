"""Writes two_point_sigmoid.json: the closed form of Eq. 1 for two points.

With two points at x=a and x=a+1 on the same row, equal sigma and no
truncation, the ratio of their Gaussian weights at column u is
exp((2(u-a)-1) / (2 sigma^2)), so Eq. 1 gives
    o(u) = c0 + (c1 - c0) * sigmoid((2(u-a)-1) / (2 sigma^2)).
The values are computed from that formula with the math module only.
"""
import json
import math
import os

a, sigma, y = 2.3, 1.7, 0.4
c0 = [0.25, -1.0, 3.5]
c1 = [0.75, 2.0, 3.5]
out = []
for u in range(6):
    t = (2 * (u - a) - 1) / (2 * sigma * sigma)
    s = 1.0 / (1.0 + math.exp(-t))
    out.append([p + (q - p) * s for p, q in zip(c0, c1)])
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "two_point_sigmoid.json"), "w") as f:
    json.dump({"source": "closed form of Eq. 1 for two points (see make_two_point_sigmoid.py)",
               "a": a, "sigma": sigma, "y": y, "c0": c0, "c1": c1, "u": list(range(6)), "out": out},
              f, indent=1)
