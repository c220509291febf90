"""Writes the hand-derived fixtures in this folder (uses only the math module).

knn_line.json -- a worked example of the common-graph construction (Sec.
  "Geodesic Sinkhorn Distances": one graph from an affinity kernel; Sec.
  "Heat Diffusion on a Graph": weighted adjacency A).  Points 0, 1, 3, 7 on a
  line, k = 1.  Nearest neighbours: 0->1 (d=1), 1->0 (d=1), 3->1 (d=2),
  7->3 (d=4); the median of the directed distances [1, 1, 2, 4] is 1.5; the
  union of directed edges is {0,1}, {1,2}, {2,3} (node ids) with squared
  lengths 1, 4, 16, so the weights are exp(-1/2.25), exp(-4/2.25), exp(-16/2.25).

two_node.json -- Algorithm 1 on one edge of unit weight with lam_hat = 2,
  mu = delta_1, nu = delta_2.  The only coupling sends all mass from node 1
  to node 2, so the value on Algorithm 1's return line is
  D = -4t ln H_12 with H_12 = (1 - exp(-2t)) / 2 (the exact heat kernel of
  the edge, eigenvalues 0 and 2).
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def knn_line():
    m = 1.5
    w01, w12, w23 = (math.exp(-d2 / (m * m)) for d2 in (1.0, 4.0, 16.0))
    adj = [[0.0, w01, 0.0, 0.0], [w01, 0.0, w12, 0.0], [0.0, w12, 0.0, w23], [0.0, 0.0, w23, 0.0]]
    return {"points": [0.0, 1.0, 3.0, 7.0], "k": 1, "median": m, "adjacency": adj,
            "source": "hand-derived; see make_golden.py docstring"}


def two_node():
    vals = {}
    for t in (0.5, 1.0, 2.0):
        vals[str(t)] = -4.0 * t * math.log((1.0 - math.exp(-2.0 * t)) / 2.0)
    return {"D_exact": vals, "source": "hand-derived; see make_golden.py docstring"}


if __name__ == "__main__":
    for name, obj in (("knn_line.json", knn_line()), ("two_node.json", two_node())):
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(obj, f, indent=1)
            f.write("\n")
