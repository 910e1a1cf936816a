"""Properties of the compiled WAVE statistic kernel that its speed depends on (CPU only: hipcc -S).

* the work fetch issues one atomic per wave (the compiler's atomic optimizer pattern: v_mbcnt to
  elect one lane), not 64 lane atomics on one address, which serialise;
* at most a few registers spilled to scratch in the FP32-arithmetic instantiations.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa") / "stat.s"
    src = os.path.join(ROOT, "paper_2510_19047_amd", "csrc", "tfsc_stat.hip")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
                           "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", src,
                           "-o", str(out)], stderr=subprocess.DEVNULL)
    return out.read_text()


def _kernels(asm, prefix):
    """(name, body up to and including its resource comment block) of each kernel whose name starts with prefix."""
    names = sorted(set(re.findall(r"^(_ZN4tfsc%d%s\w+):" % (len(prefix), prefix), asm, flags=re.M)))
    for n in names:
        start = asm.index(n + ":")
        end = asm.index("; ScratchSize:", start)
        end = asm.index("\n", end)
        yield n, asm[start:end]


def test_wave_kernel_fetch_is_one_atomic_per_wave(asm):
    found = 0
    for name, body in _kernels(asm, "k_stat_wave"):
        lines = body.splitlines()
        for i, line in enumerate(lines):
            if "global_atomic" in line:
                found += 1
                window = "\n".join(lines[max(0, i - 16):i])
                assert "v_mbcnt" in window, f"{name}: lane-wide atomic at line {i}"
    assert found >= 4


def test_wave_kernel_scratch_is_small(asm):
    """The FP32-arithmetic instantiations (every pixel store) spill at most a few registers at the
    four-waves-per-SIMD launch bound (measured faster than three waves without spills); the FP64
    validation path may spill more."""
    n = 0
    for name, body in _kernels(asm, "k_stat_wave"):
        if not re.match(r"_ZN4tfsc11k_stat_waveILi[12]Ef", name):
            continue
        n += 1
        size = int(re.search(r"; ScratchSize: (\d+)", body).group(1))
        assert size <= 64, (name, size)
    assert n >= 4


def test_multi_realisation_kernel_fetch_and_spills(asm):
    """The several-realisation kernel fetches its work the same way (one atomic per wave), and its FP32
    instantiations spill only per-chunk state, a few hundred bytes, none inside the realisation loop."""
    found = 0
    for name, body in _kernels(asm, "k_stat_wave_multi"):
        lines = body.splitlines()
        for i, line in enumerate(lines):
            if "global_atomic" in line and "_add" in line:
                found += 1
                window = "\n".join(lines[max(0, i - 16):i])
                assert "v_mbcnt" in window, f"{name}: lane-wide atomic at line {i}"
        if re.match(r"_ZN4tfsc17k_stat_wave_multiILi[12]Ef", name):
            size = int(re.search(r"; ScratchSize: (\d+)", body).group(1))
            assert size <= 320, (name, size)
    assert found >= 4


@pytest.fixture(scope="module")
def asm_vjp(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa_vjp") / "vjp.s"
    src = os.path.join(ROOT, "paper_2510_19047_amd", "csrc", "tfsc_vjp.hip")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
                           "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", src,
                           "-o", str(out)], stderr=subprocess.DEVNULL)
    return out.read_text()


def test_vjp_kernel_fetch_is_one_atomic_per_wave(asm_vjp):
    found = 0
    for name, body in _kernels(asm_vjp, "k_vjp_wave"):
        lines = body.splitlines()
        for i, line in enumerate(lines):
            if "global_atomic" in line:
                found += 1
                window = "\n".join(lines[max(0, i - 16):i])
                assert "v_mbcnt" in window, f"{name}: lane-wide atomic at line {i}"
    assert found >= 4
