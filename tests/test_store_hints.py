"""Output store hints of the compiled kernels, read from the AMD assembly of
this repository's own kernel source built for gfx950 (no GPU needed).

The plain launches (k_generate, k_fill) write their rows with non-temporal
stores at every unroll; the batch kernel (k_batch) writes with plain stores,
so that the L2 merges the partial cache lines of requests that start inside
a line.  The compiler once dropped the non-temporal hint from unroll-1 loops
(LICM promoted the store of the one-trip inner loop), which made the batch
kernel's unroll-1 shapes fast and every other unroll slow by accident; these
checks keep either choice from changing silently."""
import os
import re
import subprocess

import pytest

from paper_1108_0486_amd import build as B

pytestmark = pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not found")

PLAIN_LAUNCHES = ("_ZN2xg12_GLOBAL__N_110k_generateILj0E", "_ZN2xg12_GLOBAL__N_110k_generateILj1E",
                  "_ZN2xg12_GLOBAL__N_110k_generateILj2E", "_ZN2xg12_GLOBAL__N_16k_fillI")
BATCH = "_ZN2xg12_GLOBAL__N_17k_batchI"


@pytest.fixture(scope="module")
def inner_loop_stores(tmp_path_factory):
    """{kernel symbol: global stores inside its innermost loops}."""
    out = tmp_path_factory.mktemp("asm") / "xg_kernels.s"
    flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC")]
    subprocess.run([B.HIPCC, *flags, "--cuda-device-only", "-S", "-I", B.INCLUDE, "-I", B.CSRC,
                    os.path.join(B.CSRC, "xg_kernels.hip"), "-o", str(out)], check=True, capture_output=True)
    lines = out.read_text().split("\n")
    res = {}
    starts = [(i, m.group(1)) for i, l in enumerate(lines) if (m := re.match(r"^(_Z\S+):", l))]
    for st, name in starts:
        en = next(i for i in range(st + 1, len(lines)) if lines[i].startswith(".Lfunc_end"))
        loops = []
        for i in range(st, en):
            if "Inner Loop Header" not in lines[i]:
                continue
            j = i
            while not lines[j].startswith(".LBB"):
                j -= 1
            label = lines[j].split(":")[0]
            ends = [k for k in range(i, en)
                    if lines[k].strip().startswith(("s_cbranch", "s_branch")) and lines[k].split()[-1] == label]
            if ends:
                loops.append((j, max(ends)))
        res[name] = [lines[i].strip() for a, b in loops for i in range(a, b + 1)
                     if lines[i].strip().startswith(("global_store", "buffer_store"))]
    return res


def test_plain_launches_store_non_temporal(inner_loop_stores):
    kernels = {k: v for k, v in inner_loop_stores.items() if k.startswith(PLAIN_LAUNCHES)}
    assert len(kernels) >= 20
    for name, stores in kernels.items():
        assert stores, name
        assert all(" nt" in s for s in stores), (name, [s for s in stores if " nt" not in s])


def test_batch_kernel_stores_plain(inner_loop_stores):
    kernels = {k: v for k, v in inner_loop_stores.items() if k.startswith(BATCH)}
    assert len(kernels) == 6
    for name, stores in kernels.items():
        assert stores, name
        assert not any(" nt" in s for s in stores), (name, [s for s in stores if " nt" in s])
