"""Readers for the fixtures under tests/golden/ (values printed in the paper)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]


def table2():
    """Table 2 matrix as printed, 10 x 10 float64."""
    return np.array([[float(x) for x in ln.split()] for ln in _lines("table2_corr.txt")])


def table3():
    """Table 3: eigenvalues, variance %, cumulative % (as printed strings and
    floats) and the loadings (rows are components)."""
    sec = None
    eig, load = [], []
    for ln in _lines("table3_pca.txt"):
        if ln.startswith("["):
            sec = ln
            continue
        if sec == "[eigen]":
            eig.append(ln.split()[1:])
        else:
            load.append([float(x) for x in ln.split()])
    return {"eig_str": [e[0] for e in eig], "var_str": [e[1] for e in eig],
            "cum_str": [e[2] for e in eig],
            "eigval": np.array([float(e[0]) for e in eig]),
            "var_pct": np.array([float(e[1]) for e in eig]),
            "cum_pct": np.array([float(e[2]) for e in eig]),
            "loadings": np.array(load)}
