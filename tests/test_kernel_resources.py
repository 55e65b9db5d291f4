"""The screen kernels keep their accumulators and arguments in registers: no
kernel of screen_pairs.hip uses scratch memory or spills vector registers,
and each fits two workgroups per CU (at most 256 VGPRs, 80 KiB of LDS).
Compiles the source for gfx950 (device code only, assembly with metadata);
no GPU is needed."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1702_04739_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def screen_kernels(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_1702_04739_amd.csrc import build as B
    out = str(tmp_path_factory.mktemp("asm") / "screen_pairs.s")
    cmd = [HIPCC, *B.FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, "screen_pairs.hip"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    text = open(out).read()
    meta = text[text.find("amdhsa.kernels"):]
    kernels = {}
    for entry in re.split(r"\n  - ", meta)[1:]:
        name = re.search(r"\.name:\s+(\S+)", entry)
        if not name or "k_screen_pairs" not in name.group(1):
            continue
        get = lambda key: int(re.search(r"\.%s:\s+(\d+)" % key, entry).group(1))
        kernels[name.group(1)] = dict(vgpr=get("vgpr_count"), spill=get("vgpr_spill_count"),
                                      private=get("private_segment_fixed_size"),
                                      lds=get("group_segment_fixed_size"))
    assert len(kernels) >= 20, sorted(kernels)
    return kernels


def test_no_scratch_no_spills(screen_kernels):
    bad = {k: v for k, v in screen_kernels.items() if v["private"] or v["spill"]}
    assert not bad, bad


def test_two_workgroups_per_cu(screen_kernels):
    for k, v in screen_kernels.items():
        assert v["vgpr"] <= 256, (k, v)
        assert 2 * v["lds"] <= 160 * 1024, (k, v)
