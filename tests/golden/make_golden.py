"""Write the stored expected resultants under tests/golden/ from the oracle alone.

Usage:  python tests/golden/make_golden.py [deg6|deg20|all]

Each file holds res(f, g; y) (the Sylvester determinant of Section 2,
"Resultants" paragraph) for one seeded synthetic pair, computed by
``oracle.resultant.resultant_y`` (Bareiss over Z[x]).  The inputs are rebuilt
from ``paper_1201_1548_amd.synth`` and their digest is stored beside the
result, so a change of the generator invalidates the file loudly.

File format (text): comment lines start with '#'; then 'inputs <sha256>',
'degree <d>', and d+1 lines with the coefficients of x^0 .. x^d in decimal.
"""

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.resultant import resultant_y  # noqa: E402
from paper_1201_1548_amd import synth  # noqa: E402


def input_digest(F, G):
    return hashlib.sha256(json.dumps([F, G]).encode()).hexdigest()


def write(name, F, G, note):
    t0 = time.time()
    R = resultant_y(F, G)
    dt = time.time() - t0
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        fh.write("# res(f, g; y) in Z[x]: determinant of the Sylvester matrix (Section 2, 'Resultants').\n")
        fh.write("# written by tests/golden/make_golden.py with oracle.resultant.resultant_y only.\n")
        fh.write("# %s\n" % note)
        fh.write("# oracle time %.1f s on one core\n" % dt)
        fh.write("inputs %s\n" % input_digest(F, G))
        fh.write("degree %d\n" % (len(R) - 1))
        for c in R:
            fh.write("%d\n" % c)
    print(name, "degree", len(R) - 1, "time %.1f s" % dt, flush=True)


def load(name):
    """(digest, coefficients) of a stored golden file."""
    path = os.path.join(HERE, name)
    digest = None
    coeffs = []
    deg = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            if line.startswith("inputs "):
                digest = line.split()[1]
            elif line.startswith("degree "):
                deg = int(line.split()[1])
            elif line.strip():
                coeffs.append(int(line))
    assert deg == len(coeffs) - 1
    return digest, coeffs


def main(which):
    if which in ("deg6", "all"):
        for inst in range(4):
            F, G = synth.pair_deg6(inst)
            write("deg6_res_%d.txt" % inst, F, G,
                  "dense total degree 6, coefficients uniform in [-2^10, 2^10], instance %d" % inst)
    if which in ("deg20", "all"):
        F, G = synth.pair_deg20(0)
        write("deg20_res_0.txt", F, G, "dense total degree 20, uniform 32-bit signed coefficients, instance 0")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "deg6")
