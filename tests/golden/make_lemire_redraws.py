"""Writes lemire_redraws.txt: walkers whose injection draw hits the redraw branch of the
bucket sampler (Lemire's multiply-and-reject on 32-bit words; a rejected word is replaced by
word 0 of the block with counter (n, w, e, tag | 2^31) and key (key0, key1 ^ r) for the r-th
redraw).  Found by brute force with the oracle's own Philox4x32-10 (oracle/walker.c,
oracle_find_redraws); nothing here comes from the HIP library.

Rows of the file: n_out seed realization inject_lead walker redraws bucket.
Cases: n_out = 16138 (W = 8, L = 2017), where 2^32 mod n_out = 16114 gives a rejection
probability of 3.75e-6 per word, searched until at least one walker needs two redraws; and
n_out = 1002 (the W = 10 x L = 100 wire), single redraws.

    python tests/golden/make_lemire_redraws.py        (about 20 minutes on 8 cores)
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import walker as OW  # noqa: E402

SEED = 180510164
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lemire_redraws.txt")


def main():
    rows = []
    # single redraws: the first four walkers of each injection lead, both table sizes
    for nout, count in ((16138, 1 << 24), (1002, 1 << 28)):
        for lead in (0, 1):
            n, hits = OW.find_redraws(SEED, 0, lead, 0, 0, nout, 0, count, 1, max_out=4)
            assert n >= 4, (nout, lead, n)
            rows += [(nout, SEED, 0, lead, w, r, c) for w, r, c in hits]
    # two or more redraws at n_out = 16138: whole 2^32 walker ranges of successive realizations
    doubles = []
    r = 0
    while not doubles and r < 64:
        for lead in (0, 1):
            n, hits = OW.find_redraws(SEED, r, lead, 0, 0, 16138, 0, 1 << 32, 2, max_out=8)
            doubles += [(16138, SEED, r, lead, w, rr, c) for w, rr, c in hits]
            print(f"realization {r} lead {lead}: {n} walkers with >= 2 redraws", flush=True)
        r += 1
    assert doubles
    rows += doubles
    with open(OUT, "w") as f:
        f.write("# Walkers whose injection draw (step 0, energy index 0) needs Lemire redraws;\n")
        f.write("# written by tests/golden/make_lemire_redraws.py with the oracle's Philox.\n")
        f.write("# n_out seed realization inject_lead walker redraws bucket\n")
        for row in rows:
            f.write(" ".join(str(x) for x in row) + "\n")
    print(f"wrote {len(rows)} rows to {OUT}")


if __name__ == "__main__":
    main()
