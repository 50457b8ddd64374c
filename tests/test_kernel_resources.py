"""Resource guard of the HIP kernels (built for gfx950 on the CPU, no GPU needed).

Every device function is inlined into its kernel: no kernel makes a call (an earlier build
that called out-of-line slow paths with references to the caller's locals on the scratch stack
once faulted the GPU, see the fault notes in the design document). Scratch memory is used only
for a few register spills (no dynamic stack, at most 96 bytes per lane), and the kernels of
the camera workload keep the occupancy they are tuned for."""
import concurrent.futures as cf
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_01844_amd", "csrc")
SOURCES = ["compress.hip", "decompress.hip", "mlp.hip", "integrate.hip", "words32.hip", "capi.hip"]


def _compile(src, tmp):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    asm = os.path.join(tmp, src + ".s")
    cmd = [hipcc, "-O3", "--offload-arch=gfx950", "-std=c++17", "--cuda-device-only", "-S",
           "-Rpass-analysis=kernel-resource-usage", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-o", asm, os.path.join(CSRC, src)]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert res.returncode == 0, res.stdout[-2000:]
    with open(asm) as f:
        return res.stdout, f.read()


def _parse(remarks):
    """{function: {field: value}} from the kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in remarks.splitlines():
        if "remark:" not in line:
            continue
        body = line.split("remark:", 1)[1].split("[-Rpass", 1)[0].strip()
        if body.startswith("Function Name:"):
            cur = body.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur and ":" in body:
            k, v = body.rsplit(":", 1)
            out[cur][k.strip()] = v.strip()
    return out


@pytest.fixture(scope="module")
def resources(tmp_path_factory):
    if not os.path.exists(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    tmp = str(tmp_path_factory.mktemp("res"))
    with cf.ThreadPoolExecutor(len(SOURCES)) as pool:
        outs = list(pool.map(lambda s: _compile(s, tmp), SOURCES))
    funcs, asm = {}, ""
    for remarks, text in outs:
        funcs.update(_parse(remarks))
        asm += text
    return funcs, asm


def test_no_calls_and_no_stack_objects(resources):
    funcs, asm = resources
    assert funcs, "no kernel found"
    kernels = set(re.findall(r"^\s*\.amdhsa_kernel\s+(\S+)", asm, re.M))
    assert set(funcs) == kernels, "functions outside kernels: %s" % sorted(set(funcs) - kernels)[:5]
    assert not re.search(r"^\s*s_(swappc|setpc)_b64", asm, re.M), "a kernel makes a call"
    for name, r in funcs.items():
        assert r["Dynamic Stack"] == "False", name
        assert int(r["ScratchSize [bytes/lane]"]) <= 96, (name, r["ScratchSize [bytes/lane]"])


def test_camera_kernels_keep_their_occupancy(resources):
    funcs, _ = resources
    want = {"decompress_kernelILi2ELb0ELb0E": 5, "stats_kernelILi2ELb0ELi0E": 5, "pack_kernelILi2ELb0E": 5}
    for frag, occ in want.items():
        hits = [r for n, r in funcs.items() if frag in n]
        assert hits, frag
        assert all(int(r["Occupancy [waves/SIMD]"]) >= occ for r in hits), (frag, [r["Occupancy [waves/SIMD]"] for r in hits])
