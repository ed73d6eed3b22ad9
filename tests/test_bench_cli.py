"""Host-side checks of bench.py's contract: it refuses more than one GPU with a
message, and its carried profiler counters are well formed for every workload
they name (the kernel-source hash they are keyed on, positive byte, FLOP and
instruction counts, executed work below what the fused pass could issue)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not any(line.startswith("{") for line in r.stdout.splitlines())


def test_counters_are_well_formed():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2602_01057_amd.inputs import PRESETS
    for name, c in bench.COUNTERS.items():
        assert name in PRESETS, name
        sha = c["sources_sha256_prefix"]
        assert len(sha) == 16 and int(sha, 16) >= 0
        assert c["traffic_bytes"] > 0
        for k in ("fused", "forward"):
            assert c[k]["flops"] > 0 and c[k]["valu_insts"] > 0
            # 64 lanes per wave instruction bound the FLOPs an instruction can do
            assert c[k]["flops"] <= 64 * 2 * c[k]["valu_insts"]
        # the fused pass runs the forward's evaluation and more
        assert c["fused"]["valu_insts"] > c["forward"]["valu_insts"]
    for f in bench.KERNEL_SOURCES:
        assert os.path.isfile(os.path.join(ROOT, "paper_2602_01057_amd", "csrc", f)), f
