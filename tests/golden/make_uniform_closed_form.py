"""Writes uniform_closed_form.txt: exact objective values of the Tsallis
objective on uniform histograms, from the closed form alone (no oracle, no GPU).

Derivation (Tsallis-entropy section; the pseudo-additive composition applied
recursively for more than two classes): with p_i = 1/L, a class of m bins has
mass w = m/L and sum_i (p_i/w)^q = m^(1-q), so 1 + (1-q) S_j = m^(1-q); the
composition multiplies the factors 1 + (1-q) S_j, hence
    S(t) = ln_q(prod_j m_j) = ((prod_j m_j)^(1-q) - 1) / (1 - q).
Values are evaluated with 60-digit decimal arithmetic and printed to 17
significant digits.
"""
import itertools
import os
from decimal import Decimal, getcontext

getcontext().prec = 60
CASES = [(4, 1, "0.8"), (5, 1, "1.5"), (6, 2, "0.5"), (7, 3, "2.0"), (10, 2, "0.8")]


def ln_q(x, q):
    e = Decimal(1) - Decimal(q)
    return (Decimal(x) ** e - 1) / e


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "uniform_closed_form.txt")
    with open(out, "w") as f:
        f.write("# Tsallis objective on uniform histograms: S = ln_q(prod of class sizes).\n")
        f.write("# Source: closed form derived from the Tsallis-entropy section of\n")
        f.write("# arXiv 2012.10684 (class entropies, pseudo-additive objective);\n")
        f.write("# written by make_uniform_closed_form.py.\n")
        f.write("# columns: L k q thresholds(comma) S\n")
        for L, k, q in CASES:
            for t in itertools.combinations(range(L - 1), k):
                edges = [-1] + list(t) + [L - 1]
                m = 1
                for j in range(k + 1):
                    m *= edges[j + 1] - edges[j]
                f.write(f"{L} {k} {q} {','.join(map(str, t))} {float(ln_q(m, q))!r}\n")


if __name__ == "__main__":
    main()
