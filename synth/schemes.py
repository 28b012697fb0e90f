"""Scheme specifications: order p, step counts, which of them are free, and
the free weights as exact rationals ("num/den" strings).

The dependent weights are never stored: every consumer derives them from
these inputs through the order constraints (Sect. 3.7).
"""

# Square order-4 Richardson scheme over N = {2, 4} (Sect. 3.2, m = p/2).
SQUARE4_2_4 = dict(name="square4_2_4", p=4, steps=(2, 4), free_idx=(), c_free=())

# Order 8 over all even step counts {2,...,12} (Sect. 3.4: using every even
# count up to N_max gives the best optimised schemes), 4 dependent and 2 free
# weights.  The free weights (for N = 10 and N = 12) were produced by the
# imaginary-axis optimiser of the oracle (oracle/freeze_scheme.py writes them,
# with their exact ISB, to tests/golden/order8_k6_scheme.json; a test checks
# that these literals match that file).
ORDER8_K6 = dict(name="order8_k6", p=8, steps=(2, 4, 6, 8, 10, 12), free_idx=(4, 5),
                 c_free=("-126/23", "462/85"))

# The paper's fully determined optimum schemes (Sect. 3.3, Table 1).
FULLDET8 = dict(name="fulldet8", p=8, steps=(2, 16, 18, 20), free_idx=(), c_free=())
FULLDET12 = dict(name="fulldet12", p=12, steps=(2, 8, 12, 14, 16, 20), free_idx=(), c_free=())
FULLDET16 = dict(name="fulldet16", p=16, steps=(2, 8, 10, 12, 14, 16, 18, 22), free_idx=(),
                 c_free=())

# The paper's methods of choice (Sect. 3.8): dependent counts first, then free.
GBS_8_6 = dict(name="gbs_8_6", p=8, steps=(2, 4, 6, 10, 8, 12, 14, 16, 18, 20, 22),
               free_idx=tuple(range(4, 11)),
               c_free=("2165/767488", "13805/611712", "4553/72080", "14503/66520",
                       "27058/7627", "-86504/5761", "40916/3367"))
# The printed n_free list lacks the 24 that the eleven printed weights need.
GBS_8_8 = dict(name="gbs_8_8", p=8,
               steps=(2, 26, 28, 30, 4, 6, 8, 10, 12, 14, 16, 18, 20, 22, 24),
               free_idx=tuple(range(4, 15)),
               c_free=("6833/476577792", "10847/91078656", "15235/34643968", "383/321152",
                       "543/198784", "9947/1741056", "6243/543104", "6875/296192",
                       "1401/28496", "17713/152688", "6375/19264"))
GBS_12_8 = dict(name="gbs_12_8", p=12,
                steps=(2, 8, 10, 16, 24, 26, 4, 6, 12, 14, 18, 20, 22, 28, 30),
                free_idx=tuple(range(6, 15)),
                c_free=("235/21030240256", "4147/1612709888", "11521/39731200", "2375/3528704",
                        "6435/708736", "1291/15780", "11311/4672", "-180864/751",
                        "222080/2079"))

ALL = [SQUARE4_2_4, ORDER8_K6, FULLDET8, FULLDET12, FULLDET16, GBS_8_6, GBS_8_8, GBS_12_8]


def free_as_pairs(scheme):
    """c_free as (numerator, denominator) integer pairs."""
    out = []
    for s in scheme["c_free"]:
        num, den = s.split("/")
        out.append((int(num), int(den)))
    return out
