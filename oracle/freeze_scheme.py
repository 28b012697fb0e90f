"""Writes tests/golden/order8_k6_scheme.json: the free weights of the order-8
scheme over N = {2,...,12} with N = 10, 12 free (test infrastructure only).

Steps (App. B and Sect. 3.8): bisection over the covered segment with the
convex minimax inner problem; a weighted-slack re-solve just below the optimum
to keep |R| < 1 off the origin; rationalisation to denominators <= 100; the
exact ISB of the rational scheme.  Run:  python -m oracle.freeze_scheme
"""
import json
import os

from . import optimize, stability, weights

P, STEPS, FREE = 8, [2, 4, 6, 8, 10, 12], [4, 5]


def freeze():
    y_star, _ = optimize.optimise(P, STEPS, FREE, tol=1e-4)
    _, cf = optimize.robust(P, STEPS, FREE, y_star)
    cr = optimize.rationalise(cf, max_den=100)
    c = weights.weights(P, STEPS, FREE, cr)
    isb = stability.isb(stability.extrapolated_poly(STEPS, c))
    return dict(p=P, steps=STEPS, free_idx=FREE,
                c_free=["%d/%d" % (x.numerator, x.denominator) for x in cr],
                lp_isb=y_star, exact_isb=isb, isb_n=isb / (max(STEPS) + 1))


if __name__ == "__main__":
    out = freeze()
    path = os.path.join(os.path.dirname(__file__), "..", "tests", "golden",
                        "order8_k6_scheme.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))
