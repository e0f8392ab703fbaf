"""Register budgets of the kernel builds, read from the compiler (no GPU).

The host launches no kernel build that uses private (scratch) memory; it
checks each build's private segment at batch creation and sends the RVEs of
an excluded build to the next build that holds them, else to the streamed
kernel.  This test pins which builds the compiler leaves with a private
segment, so a change that makes a launched build spill fails here, on the
CPU, before it reaches a GPU: every build outside the list below must have
zero scratch bytes per lane.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_09427_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-I", os.path.join(ROOT, "include"), "--cuda-device-only",
         "-Rpass-analysis=kernel-resource-usage"]

# builds with a private segment, each excluded at run time by the host
# (FP64 state of 4+2 slots per thread does not fit 168 or 128 VGPRs; the
# FP64 streamed kernel in 128; the lean 1024-thread tangent task with 8 node
# slots).  The FP32 6+3 slot builds fit 128 VGPRs with the inverse mass
# held in the LDS position record.
EXPECTED_PRIVATE = {
    "dr_resident_kernel<double, 768, 4, 2, false>", "dr_resident_kernel<double, 768, 4, 2, true>",
    "dr_resident_kernel<double, 1024, 4, 2, false>", "dr_resident_kernel<double, 1024, 4, 2, true>",
    "dr_resident_kernel<double, 1024, 6, 3, false>", "dr_resident_kernel<double, 1024, 6, 3, true>",
    "dr_streamed_kernel<double, 1024, false>", "dr_streamed_kernel<double, 1024, true>",
    "cg_res_kernel<false, 1024, 8, true>", "cg_res_kernel<true, 1024, 8, true>",
}


def kernel_resources(src):
    out = subprocess.run([HIPCC, *FLAGS, "-c", src, "-o", os.devnull], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr[-2000:]
    rows, cur = [], None
    for line in out.stderr.splitlines():
        m = re.search(r"remark: (.*?) \[-Rpass", line)
        if not m:
            continue
        t = m.group(1)
        if t.startswith("Function Name:"):
            cur = {"name": t.split(":", 1)[1].strip()}
            rows.append(cur)
        elif cur is not None and ":" in t:
            k, v = t.split(":", 1)
            cur[k.strip()] = v.strip()
    names = subprocess.run(["c++filt"], input="\n".join(r["name"] for r in rows), capture_output=True,
                           text=True).stdout.splitlines()
    res = {}
    for r, n in zip(rows, names):
        n = re.sub(r"\(.*\)$", "", n.replace("rve::", "").replace("(anonymous namespace)::", "")).strip()
        n = re.sub(r"^void ", "", n)
        res[n] = int(r.get("ScratchSize [bytes/lane]", "0"))
    return res


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_only_the_excluded_builds_use_private_memory():
    private = set()
    seen = 0
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip"):
            res = kernel_resources(os.path.join(CSRC, f))
            seen += len(res)
            private |= {n for n, b in res.items() if b > 0}
    assert seen > 40
    assert private == EXPECTED_PRIVATE, (sorted(private - EXPECTED_PRIVATE), sorted(EXPECTED_PRIVATE - private))
