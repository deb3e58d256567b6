"""Writes the stored expected values used by the GPU tests.  Calls only the
CPU oracle (exact transfer matrix) on the seeded inputs of `instances`.

    python tests/golden/make_golden.py            # every table
    python tests/golden/make_golden.py sg32x24    # one table
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import instances as I  # noqa: E402
from oracle import tm, tm_c, value  # noqa: E402


def larger():
    """Exact pins for larger parity cases (C transfer matrix, multiword
    counts)."""
    with open(os.path.join(HERE, "sg20.txt"), "w") as f:
        f.write("# +-J spin glass 20x20 open lattice, zero field, seeds 0-4:\n")
        f.write("# seed E0 degeneracy  (oracle: exact transfer matrix, C)\n")
        for s in range(5):
            g = I.spin_glass_square(20, s)
            e0, deg = tm_c.spin_glass_lattice(20, 20, g["edges"], g["J"])
            f.write("%d %d %d\n" % (s, e0, deg))
            f.flush()
    with open(os.path.join(HERE, "ksg20.txt"), "w") as f:
        f.write("# unweighted MIS on King's subgraph 20x20, fill 0.8, seeds 0-4:\n")
        f.write("# seed n W* count  (oracle: exact transfer matrix, C)\n")
        for s in range(5):
            g = I.kings_subgraph(20, s)
            w, c = tm_c.kings_subgraph(g)
            f.write("%d %d %d %d\n" % (s, g["n"], w, c))
            f.flush()
    with open(os.path.join(HERE, "sg24.txt"), "w") as f:
        f.write("# +-J spin glass 24x24 open lattice, zero field, seeds 0-1:\n")
        f.write("# seed E0 degeneracy  (oracle: exact transfer matrix, C)\n")
        for s in range(2):
            g = I.spin_glass_square(24, s)
            e0, deg = tm_c.spin_glass_lattice(24, 24, g["edges"], g["J"])
            f.write("%d %d %d\n" % (s, e0, deg))
            f.flush()


def sg32x24():
    """+-J spin glass on a 32 x 24 open lattice (rows x columns), seeds 0-1:
    parity cases whose leaves reach 2^22 entries (C transfer matrix over the
    24-column frontier)."""
    with open(os.path.join(HERE, "sg32x24.txt"), "w") as f:
        f.write("# +-J spin glass 32x24 open lattice (32 rows, 24 columns), zero field, seeds 0-1:\n")
        f.write("# seed E0 degeneracy  (oracle: exact transfer matrix, C)\n")
        for s in range(2):
            g = I.spin_glass_rect(32, 24, s)
            e0, deg = tm_c.spin_glass_lattice(32, 24, g["edges"], g["J"])
            f.write("%d %d %d\n" % (s, e0, deg))
            f.flush()


def strips():
    """+-J spin glass strips as long as the 48x48 and 64x64 lattices (48x20
    and 64x16, rows x columns), seeds 0-1: exact values for parity cases of
    branching along the long dimension (C transfer matrix over the narrow
    frontier)."""
    for Lr, Lc in ((48, 20), (64, 16)):
        with open(os.path.join(HERE, "sg%dx%d.txt" % (Lr, Lc)), "w") as f:
            f.write("# +-J spin glass %dx%d open lattice (%d rows, %d columns), zero field, "
                    "seeds 0-1:\n" % (Lr, Lc, Lr, Lc))
            f.write("# seed E0 degeneracy  (oracle: exact transfer matrix, C)\n")
            for s in range(2):
                g = I.spin_glass_rect(Lr, Lc, s)
                e0, deg = tm_c.spin_glass_lattice(Lr, Lc, g["edges"], g["J"])
                f.write("%d %d %d\n" % (s, e0, deg))
                f.flush()


def _values(name, header, rows):
    with open(os.path.join(HERE, name), "w") as f:
        f.write(header)
        for row in rows:
            f.write(" ".join(str(x) for x in row) + "\n")
            f.flush()


def sg_values(L, seeds):
    """Ground energies of L x L +-J lattices (zero field) by the matching
    oracle; the degeneracy is beyond every exact oracle here."""
    def rows():
        for s in seeds:
            g = I.spin_glass_square(L, s)
            yield (s, value.spin_glass_planar_e0(L, g["edges"], g["J"]))
    _values("sg%d_values.txt" % L,
            "# +-J spin glass %dx%d open lattice, zero field, seeds %d-%d:\n"
            "# seed E0  (oracle: minimum-weight perfect matching on the dual)\n"
            % (L, L, seeds[0], seeds[-1]), rows())


def ksg_values(L, seeds):
    """Maximum independent set sizes of L x L King's subgraphs (fill 0.8) by
    the integer-programming oracle."""
    def rows():
        for s in seeds:
            g = I.kings_subgraph(L, s)
            yield (s, g["n"], value.mwis_milp(g["n"], g["edges"]))
    _values("ksg%d_values.txt" % L,
            "# unweighted MIS on King's subgraph %dx%d, fill 0.8, seeds %d-%d:\n"
            "# seed n W*  (oracle: integer program, HiGHS)\n"
            % (L, L, seeds[0], seeds[-1]), rows())


def sg32_values():
    sg_values(32, list(range(20)))


def ksg40_values():
    ksg_values(40, list(range(20)))


def sg48_values():
    sg_values(48, [0, 1])


def ksg64_values():
    ksg_values(64, [0, 1])


def sg16_more():
    """Further 16x16 seeds (20-319) for throughput runs over many distinct
    instances (C transfer matrix)."""
    with open(os.path.join(HERE, "sg16_more.txt"), "w") as f:
        f.write("# +-J spin glass 16x16 open lattice, zero field, seeds 20-319:\n")
        f.write("# seed E0 degeneracy  (oracle: exact transfer matrix, C)\n")
        for s in range(20, 320):
            g = I.spin_glass_square(16, s)
            e0, deg = tm_c.spin_glass_lattice(16, 16, g["edges"], g["J"])
            f.write("%d %d %d\n" % (s, e0, deg))
            f.flush()


def main():
    sg32_values()
    ksg40_values()
    sg48_values()
    ksg64_values()
    larger()
    sg32x24()
    strips()
    sg16_more()
    with open(os.path.join(HERE, "sg16.txt"), "w") as f:
        f.write("# +-J spin glass 16x16 open lattice, zero field, seeds 0-19:\n")
        f.write("# seed E0 degeneracy  (oracle: exact transfer matrix)\n")
        for s in range(20):
            e0, deg = tm.spin_glass_square(I.spin_glass_square(16, s))
            f.write("%d %d %d\n" % (s, e0, deg))
            f.flush()
    with open(os.path.join(HERE, "ksg16.txt"), "w") as f:
        f.write("# unweighted MIS on King's subgraph 16x16, fill 0.8, seeds 0-4:\n")
        f.write("# seed n W* count  (oracle: exact transfer matrix)\n")
        for s in range(5):
            g = I.kings_subgraph(16, s)
            w, c = tm.kings_subgraph(g)
            f.write("%d %d %d %d\n" % (s, g["n"], w, c))
            f.flush()


if __name__ == "__main__":
    if len(sys.argv) > 1:
        globals()[sys.argv[1]]()  # one table, e.g. sg32x24
    else:
        main()
