"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Calls only oracle/ (never the HIP path).  Run from the repository root:
    python tests/golden/make_golden.py
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


if __name__ == "__main__":
    main()
