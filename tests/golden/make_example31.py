"""Writes example31.json: concrete numbers for the worked example of §3.2.1
(Example 3.1) of the paper.

The example fixes only inequalities between its constants: A = [c1 v1, c2 v2, c3 v3]
with c1 > c2 > c3 > 0 and v1, v2, v3 orthonormal, a single recycled sketch vector
g = d2 v2 + d3 v3 with d2 > d3 > 0, v2(2) > v2(1) > v2(3) > 0 and v1(2) = v3(2) > 0.
It then prints, as formulas, the sketched residual before the first iteration,
g^T A = [0, c2 d2, c3 d3], and after the first iteration (column 2, row 2 selected),
[-c1 d2 v1(2) / v2(2), 0, c3 d3 - c3 d2 v3(2) / v2(2)], and states that the first
iteration selects column 2 and row 2 and the second selects column 1.

This script picks constants that satisfy those inequalities and evaluates the
paper's two printed formulas; it does not call the oracle.  Indices in the JSON are
0-based (paper's column 2 -> 1).
"""
import json
import os

import numpy as np


def build():
    c = np.array([3.0, 2.0, 1.0])
    d2, d3 = 0.9, 0.4
    v2 = np.array([0.55, 0.75, 0.37])
    v2 /= np.linalg.norm(v2)
    # orthonormal basis (e1, e2) of the plane orthogonal to v2
    e1 = np.array([1.0, 0.0, 0.0]) - v2[0] * v2
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(v2, e1)
    # rotate inside that plane so that v1(2) = v3(2) (second entries, 0-based index 1)
    theta = np.arctan2(e2[1] - e1[1], e1[1] + e2[1])
    v1 = np.cos(theta) * e1 + np.sin(theta) * e2
    v3 = -np.sin(theta) * e1 + np.cos(theta) * e2
    if v1[1] < 0:
        v1, v3 = -v1, -v3
    V = np.stack([v1, v2, v3], axis=1)
    assert np.allclose(V.T @ V, np.eye(3), atol=1e-14)
    assert abs(v1[1] - v3[1]) < 1e-14 and v1[1] > 0
    assert v2[1] > v2[0] > v2[2] > 0
    A = V * c[None, :]
    g = d2 * v2 + d3 * v3
    before = [0.0, c[1] * d2, c[2] * d3]
    after = [-c[0] * d2 * v1[1] / v2[1], 0.0, c[2] * d3 - c[2] * d2 * v3[1] / v2[1]]
    # the example's claimed selections follow from these numbers
    assert np.argmax(np.abs(before)) == 1
    assert np.argmax(np.abs(after)) == 0
    return {
        "source": "arXiv 2509.21963, Section 3.2.1, Example 3.1 (the two sketched "
                  "residual vectors are the paper's printed formulas evaluated at the "
                  "constants below)",
        "A": A.tolist(),
        "g": g.tolist(),
        "c": c.tolist(),
        "d": [d2, d3],
        "v": V.T.tolist(),
        "sketched_residual_before": before,
        "sketched_residual_after_iter1": after,
        "iter1_column": 1,
        "iter1_row": 1,
        "iter2_column": 0,
    }


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "example31.json")
    with open(path, "w") as f:
        json.dump(build(), f, indent=1)
    print("wrote", path)
