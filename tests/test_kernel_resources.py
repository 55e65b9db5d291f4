"""Every kernel of the library keeps its working set in registers and LDS: no
kernel uses scratch memory or spills vector registers, and each screen kernel
fits two workgroups per CU (at most 256 VGPRs, 80 KiB of LDS).  Compiles the
sources for gfx950 (device code only, assembly with its metadata); no GPU is
needed."""
import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1702_04739_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _kernels(asm):
    meta = asm[asm.find("amdhsa.kernels"):]
    out = {}
    for entry in re.split(r"\n  - ", meta)[1:]:
        name = re.search(r"\.name:\s+(\S+)", entry)
        if not name:
            continue
        get = lambda key: int(re.search(r"\.%s:\s+(\d+)" % key, entry).group(1))
        out[name.group(1)] = dict(vgpr=get("vgpr_count"), spill=get("vgpr_spill_count"),
                                  private=get("private_segment_fixed_size"), lds=get("group_segment_fixed_size"))
    return out


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_1702_04739_amd.csrc import build as B
    tmp = tmp_path_factory.mktemp("asm")

    def compile_one(src):
        out = str(tmp / (src + ".s"))
        r = subprocess.run([HIPCC, *B.FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out],
                           capture_output=True, text=True)
        assert r.returncode == 0, (src, r.stderr[-3000:])
        return _kernels(open(out).read())

    with ThreadPoolExecutor(max_workers=4) as ex:
        found = {}
        for d in ex.map(compile_one, B.SOURCES):
            found.update(d)
    assert sum("k_screen_pairs" in k for k in found) >= 20, sorted(found)
    return found


def test_no_scratch_no_spills(kernels):
    bad = {k: v for k, v in kernels.items() if v["private"] or v["spill"]}
    assert not bad, bad


def test_screen_fits_two_workgroups_per_cu(kernels):
    for k, v in kernels.items():
        if "k_screen_pairs" in k:
            assert v["vgpr"] <= 256, (k, v)
            assert 2 * v["lds"] <= 160 * 1024, (k, v)
