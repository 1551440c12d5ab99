"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Calls only oracle/ (never the HIP path).  Run from the repository root:
    python tests/golden/make_golden.py               (every file)
    python tests/golden/make_golden.py huge_skips    (the large-skip states only)
"""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402


def digest(a):
    return hashlib.sha256(a.tobytes()).hexdigest()


def main():
    lines = ["# Single xorgens stream, w = 32, (r,s,a,b,c,d) = (128,65,15,14,12,17),",
             "# omega = 0x9E3779B9, gamma = 16, seeded from 64-bit seed 42 (INIT-v1),",
             "# first 2^20 uint32 outputs.  Written by tests/golden/make_golden.py from",
             "# the CPU oracle alone.",
             ]
    st = O.OracleStreams(42, 1)
    u = st.u32(1 << 20)[0]
    lines.append("sha256_le_u32 %s" % digest(u))
    lines.append("first8 %s" % " ".join("0x%08x" % v for v in u[:8]))
    lines.append("last 0x%08x" % u[-1])
    lines.append("final_weyl 0x%08x" % st.weyl[0])
    lines.append("final_ring_sha256 %s" % digest(st.ring[0]))
    with open(os.path.join(HERE, "single_stream_seed42_2p20.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")

    lines = ["# 1024 streams, stream i seeded from 42 + i (INIT-v1), 2^20 uint32 each:",
             "# sha256 of each sampled stream's outputs (little-endian uint32).",
             "# Written by tests/golden/make_golden.py from the CPU oracle alone."]
    for i in [0, 1, 2, 511, 512, 1000, 1023]:
        one = O.OracleStreams(42 + i, 1)
        lines.append("stream %d %s" % (i, digest(one.u32(1 << 20)[0])))
    with open(os.path.join(HERE, "bulk_1024x2p20_samples.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


# Large skips whose expected states come from the oracle's matrix form: the
# x-part's one-step bit matrix T raised to J by binary powering and applied to
# the start state (no jump polynomial on either side).
HUGE_SKIPS = [
    # (name, params, seed, count, stream indices, J values)
    ("r128_w32", O.PAPER, 7, 5, range(5), [2**32 + 5, 2**50 + 3, 2**63 + 1]),
    ("r64_w32", O.R64, 21, 7, range(1, 6), [2**40 + 5, 2**63 + 1]),
    ("r64_w64", O.W64, 21, 7, range(1, 6), [2**40 + 5, 2**63 + 1]),
]


def huge_skips():
    import numpy as np
    lines = ["# x-part rings after skipping J words, by the oracle's matrix form",
             "# (T^J by binary powering of the one-step bit matrix, applied to the",
             "# seeded ring).  One line per (member, J, stream): sha256 of the ring's",
             "# little-endian words.  Written by tests/golden/make_golden.py from",
             "# the CPU oracle alone."]
    for name, p, seed, count, idx, Js in HUGE_SKIPS:
        if p.w == 64:
            ref = O.OracleStreams64(seed, count, p)
        else:
            ref = O.OracleStreams(seed, count, params=p)
        M = O.xpart_matrix(p)
        idx = list(idx)
        vs = np.stack([O.ring_to_bits(p, ref.ring[i]) for i in idx for _ in Js])
        got = O.mat_pow_apply_many(M, p.n, [J for _ in idx for J in Js], vs)
        for a, i in enumerate(idx):
            for b, J in enumerate(Js):
                ring = O.bits_to_ring(p, got[a * len(Js) + b])
                lines.append("%s seed %d stream %d J %d ring %s" % (name, seed, i, J, digest(ring)))
    with open(os.path.join(HERE, "huge_skips_matrix_form.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1:] == ["huge_skips"]:
        huge_skips()
    else:
        main()
        huge_skips()
