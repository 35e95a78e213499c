"""Register and scratch budget of every kernel in the built library, read from
its gfx950 code objects (no GPU needed).

The streaming kernels run 1024 workgroups of 256 threads across 256 compute
units, four workgroups per CU, which needs four waves per SIMD (the p(l)-CG
sweeps beyond the memory-side cache run up to six per CU where their registers
allow, chosen at run time from the kernel's occupancy); the resident
kernels run one workgroup of 1024 threads on one CU, which needs the same.  A
CDNA SIMD holds 512 registers per lane for its waves, so every kernel must stay
within 128 vector registers (arch VGPRs + AGPRs), and none may spill vector
registers or use scratch memory.  A sweep past that budget does not fail, it
runs at half occupancy or less: that has happened when values were held for
early loads (an FP32-stored sweep's preload took it to 171 registers and made
it 45 % slower), so it is checked at build time.

One exception, measured and kept: the FP32-stored l = 8 sweeps with paired x
updates hold 131-134 registers (four values per thread and vector, nine
products, the x and both p buffers) and run three waves per SIMD; holding the
compiler to four waves (amdgpu_waves_per_eu(4)) made it spill 6-20 registers
of those sweeps to scratch memory instead.  And the batch tick kernel calls
its per-slot owner step as a function, whose frame saves a callee-saved
register in 16 bytes of scratch once per slot and tick (outside the streaming
loop)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"
MAX_VGPRS = 128
# FP32-stored (f) l = 8 sweeps with paired x updates (last template flag true)
EXCEPTION = re.compile(r"_ZN4plcg\d+plcg_(var_|diag_|csr_)?sweep_kernelILi8E(Lb[01]E)?fLi\d+ELb1EE")
MAX_EXCEPTION = 136
CALL_FRAME = ("_ZN4plcg17batch_tick_kernel", 16)

pytestmark = pytest.mark.skipif(
    not all(os.path.exists(os.path.join(LLVM, t))
            for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")),
    reason="ROCm LLVM tools not available")


def _kernels(tmp_path):
    """(name, metadata dict) of every kernel in every gfx950 code object."""
    from paper_1905_06850_amd import plcg
    fat = tmp_path / "fat.bin"
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}",
                    plcg.LIB_PATH, os.devnull], check=True, capture_output=True)
    data = fat.read_bytes()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)]
    assert starts, "no offload bundles in .hip_fatbin"
    out = []
    for k, s in enumerate(starts):
        e = starts[k + 1] if k + 1 < len(starts) else len(data)
        b = tmp_path / f"bundle{k}.bin"
        b.write_bytes(data[s:e])
        co = tmp_path / f"co{k}.o"
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                        f"--input={b}", f"--targets={TARGET}", f"--output={co}"],
                       check=True, capture_output=True)
        notes = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", str(co)],
                               check=True, capture_output=True, text=True).stdout
        # one metadata map per kernel, each starting with `- .agpr_count:`
        for block in re.split(r"\n\s+- \.agpr_count:", notes)[1:]:
            block = ".agpr_count:" + block
            fields = dict(re.findall(r"^\s*\.?([\w]+):\s+(\S+)\s*$", block, re.M))
            name = fields.get("name")
            if name and name.startswith("_Z"):
                out.append((name, fields))
    return out


def test_every_kernel_fits_four_waves_per_simd(tmp_path):
    ks = _kernels(tmp_path)
    names = [n for n, _ in ks]
    # all five translation units are there
    for part in ("plcg_sweep_kernel", "cg_sweep_a_kernel", "var_", "resident_kernel",
                 "batch_tick_kernel"):
        assert any(part in n for n in names), part
    over = []
    for name, f in ks:
        v = int(f["vgpr_count"]) + int(f.get("agpr_count", 0))
        spill = int(f.get("vgpr_spill_count", 0))
        scratch = int(f.get("private_segment_fixed_size", 0))
        if name.startswith(CALL_FRAME[0]) and scratch <= CALL_FRAME[1]:
            scratch = 0
        limit = MAX_EXCEPTION if EXCEPTION.match(name) else MAX_VGPRS
        if v > limit or spill or scratch:
            over.append((name, v, spill, scratch))
    assert not over, over
    assert any(EXCEPTION.match(n) for n in names)


def test_fp32_sweeps_use_no_more_registers_than_twice_their_fp64_form(tmp_path):
    """A sweep stored in FP32 handles four values per thread and vector to the
    FP64 sweep's two, so it may use more registers, but not more than twice."""
    regs = {}
    for name, f in _kernels(tmp_path):
        m = re.match(r"_ZN4plcg17plcg_sweep_kernelIL(.*)EEvNS_10SweepArgsT", name)
        if m:
            regs[m.group(1)] = int(f["vgpr_count"])
    pairs = 0
    for key, v in regs.items():
        if "Ef" in key:
            d = regs.get(key.replace("Ef", "Ed", 1))
            if d is not None:
                pairs += 1
                assert v <= 2 * d, (key, v, d)
    assert pairs > 0
