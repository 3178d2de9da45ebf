"""CPU checks of the build flags and of the native sources' hardware rules.

* The library is built for gfx950 only, with packed FP32 instructions disabled.
* Inline assembly is limited to an allow-list of mnemonics (the LDS barrier).
  Packed FP32 arithmetic and memory writes are left to the compiler.
* No stream priorities, host registration of existing memory or uncached
  allocations.  No platform-compatibility branches.
* hipMemsetAsync appears only outside graph capture: the batch solver's
  captured sequence clears memory with kernels.
"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2301_08911_amd", "csrc")
ALLOWED_ASM = {"s_waitcnt", "s_barrier"}


def sources():
    out = {}
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".cpp", ".hpp", ".h")):
            out[f] = open(os.path.join(CSRC, f)).read()
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        out["include/" + f] = open(os.path.join(ROOT, "include", f)).read()
    return out


def test_build_flags_target_gfx950_without_packed_fp32():
    from paper_2301_08911_amd import build
    flags = build.FLAGS
    archs = [f for f in flags if f.startswith("--offload-arch")]
    assert archs == ["--offload-arch=gfx950"]
    i = flags.index("-packed-fp32-ops")
    assert flags[i - 3:i] == ["-Xclang", "-target-feature", "-Xclang"]


def test_inline_asm_uses_only_allowed_mnemonics():
    seen = set()
    for name, text in sources().items():
        # every asm statement must be one this parser reads
        assert len(re.findall(r"\basm\b", text)) == len(re.findall(
            r"\basm\s*(?:volatile\s*)?\(\s*\"", text)), name
        for m in re.finditer(r"\basm\s*(?:volatile\s*)?\(\s*((?:\"[^\"]*\"\s*)+)", text):
            body = "".join(re.findall(r"\"([^\"]*)\"", m.group(1)))
            for line in re.split(r"\\n|\\t|;", body):
                op = line.strip().split()[0] if line.strip() else None
                if op is not None:
                    assert op in ALLOWED_ASM, (name, op)
                    seen.add(op)
    assert seen == ALLOWED_ASM


def test_no_priority_streams_host_registration_or_uncached_memory():
    banned = ["StreamCreateWithPriority", "HostRegister", "DeviceMallocUncached",
              "ExtMallocWithFlags", "__HIP_PLATFORM", "__CUDA_ARCH__", "hipify"]
    for name, text in sources().items():
        for b in banned:
            assert b not in text, (name, b)


def test_memset_only_outside_graph_capture():
    # The one hipMemsetAsync clears the density-check flag in set_density, which
    # synchronizes its stream and so never runs under capture.
    hits = [(name, m.start()) for name, text in sources().items()
            for m in re.finditer(r"hipMemsetAsync", text)]
    assert len(hits) == 1 and hits[0][0] == "solver.cpp", hits
    text = open(os.path.join(CSRC, "solver.cpp")).read()
    head = text[:hits[0][1]]
    fn = head[head.rfind("Status "):]
    assert fn.startswith("Status set_density("), fn[:60]
    assert "hipStreamSynchronize" in text[hits[0][1]:hits[0][1] + 800]
