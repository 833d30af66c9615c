"""Properties of the gfx950 code of the hot kernels that their speed depends on (CPU only: the
kernels are compiled to assembly here, nothing runs).

- The split BF16 contraction copies its operand stages into LDS with buffer loads.  With
  global_load_lds copies in flight, the compiler cannot use the in-order completion of LDS
  reads and opens every K step with a full LDS wait; with buffer loads, only the stage
  barrier's wait drains everything.
- The contraction and generation kernels spill no vector registers.
- Generation writes its bitmasks with global (not flat) stores: a flat access also counts
  against the LDS counter.
"""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_07642_amd", "csrc")

SPLIT = "_ZN2rr15contract_kernelILi0ELi8ELi2ELi2ELi4ELb0EEEvNS_12ContractArgsE"      # split, S = 4
SPLIT_BATCH = "_ZN2rr15contract_kernelILi0ELi8ELi2ELi2ELi4ELb1EEEvNS_12ContractArgsE"
GEN = "_ZN2rr10gen_kernelILi4ELb0EEEvNS_7GenArgsE"
GEN_BATCH = "_ZN2rr16gen_batch_kernelILi4EEEvPKNS_7GenArgsEmm"


def _asm(src, tmp_path):
    from paper_2501_07642_amd import build
    hipcc = build.hipcc()
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    out = tmp_path / (os.path.splitext(src)[0] + ".s")
    flags = [f for f in build.flags() if f != "-fPIC"]
    r = subprocess.run([hipcc, *flags, "-I", CSRC, "--cuda-device-only", "-S", os.path.join(CSRC, src),
                        "-o", str(out)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


def _body(asm, name):
    i = asm.index(name + ":")
    return asm[i:asm.index(".Lfunc_end", i)]


def _meta(asm, name, key):
    """A field of the kernel's metadata record (the fields after .name, up to the next record)."""
    i = asm.index(".name:           " + name + "\n")
    j = asm.find("- .agpr_count", i)
    m = re.search(r"\." + key + r":\s+(\d+)", asm[i:j if j > 0 else len(asm)])
    return int(m.group(1))


def _main_loop(body):
    """The basic block holding the most MFMA instructions."""
    blocks = re.split(r"^\.LBB\S+:", body, flags=re.M)
    return max(blocks, key=lambda b: b.count("v_mfma"))


@pytest.fixture(scope="module")
def contract_asm(tmp_path_factory):
    return _asm("rr_contract.hip", tmp_path_factory.mktemp("isa"))


@pytest.fixture(scope="module")
def gen_asm(tmp_path_factory):
    return _asm("rr_gen.hip", tmp_path_factory.mktemp("isa"))


@pytest.mark.parametrize("name", [SPLIT, SPLIT_BATCH])
def test_split_contraction_waits_only_at_the_stage_barrier(contract_asm, name):
    body = _body(contract_asm, name)
    assert "global_load_lds" not in body
    assert re.search(r"buffer_load_dwordx4 .* lds", body)
    loop = _main_loop(body)
    assert loop.count("v_mfma_f32_32x32x16_bf16") == 64          # one LDS stage: 8 K steps x 8 MFMA
    full = re.findall(r"s_waitcnt (?:vmcnt\(0\) expcnt\(0\) )?lgkmcnt\(0\)$", loop, flags=re.M)
    assert len(full) <= 2, full                                  # the stage barrier (+ the loop head)
    assert "v_readfirstlane" not in loop                         # no per-load uniformity loops
    assert _meta(contract_asm, name, "vgpr_spill_count") == 0


@pytest.mark.parametrize("name", [GEN, GEN_BATCH])
def test_generation_stores_are_global(gen_asm, name):
    body = _body(gen_asm, name)
    assert not re.search(r"^\s*flat_", body, flags=re.M)
    assert re.search(r"global_store_dwordx4 .* nt", body)
    assert _meta(gen_asm, name, "vgpr_spill_count") == 0
