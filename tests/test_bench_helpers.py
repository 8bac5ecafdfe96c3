"""Host logic of bench.py that decides whether a committed counter summary still
describes the current kernel source.  CPU only; works on copies in a temporary tree."""
import importlib.util
import json
import os
import shutil

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture
def bench(tmp_path):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    csrc = tmp_path / "paper_2605_12085_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("forward.hip", "backproject.hip", "device_util.h", "common.h", "plan.hip"):
        shutil.copy(os.path.join(ROOT, "paper_2605_12085_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    mod.ROOT = str(tmp_path)
    return mod, tmp_path


def test_hash_ignores_comments_and_spacing(bench):
    mod, root = bench
    h0 = mod.kernel_source_hash("fp_kernel")
    p = root / "paper_2605_12085_amd" / "csrc" / "forward.hip"
    text = p.read_text()
    p.write_text("// a new leading comment\n/* and a block\n   comment */\n" + text.replace("\n", "\n\n", 5))
    assert mod.kernel_source_hash("fp_kernel") == h0
    p.write_text(text.replace("constexpr int kRows = 16;", "constexpr int kRows = 8;"))
    assert mod.kernel_source_hash("fp_kernel") != h0


@pytest.mark.parametrize("shared", ["device_util.h", "common.h", "plan.hip"])
def test_hash_covers_the_shared_sources(bench, shared):
    # device helpers, shared declarations and the host code that picks launch shapes
    mod, root = bench
    h_fp, h_bp = mod.kernel_source_hash("fp_kernel"), mod.kernel_source_hash("bp_kernel")
    p = root / "paper_2605_12085_amd" / "csrc" / shared
    p.write_text(p.read_text() + "\nnamespace fbl { constexpr int kUnused = 1; }\n")
    assert mod.kernel_source_hash("fp_kernel") != h_fp
    assert mod.kernel_source_hash("bp_kernel") != h_bp


def test_traffic_only_for_the_source_it_was_taken_on(bench):
    mod, root = bench
    rec = {"hbm_bytes_per_launch": 123456789, "kernel_source_hash": mod.kernel_source_hash("bp_kernel")}
    (root / "profiles" / "bp_kernel_c2_pmc.json").write_text(json.dumps(rec))
    assert mod.measured_traffic("bp_kernel", "c2") == 123456789
    assert mod.measured_traffic("fp_kernel", "c2") is None          # no summary
    rec["kernel_source_hash"] = "0" * 16
    (root / "profiles" / "bp_kernel_c2_pmc.json").write_text(json.dumps(rec))
    assert mod.measured_traffic("bp_kernel", "c2") is None          # taken on other code


def test_valu_issue_peak(bench):
    # 256 CUs, each issuing one wave64 VALU instruction per clock at 2.4 GHz (no packed FP32):
    # 39.3 T lane operations per second, 78.6 TFLOP/s with an FMA counted as two
    mod, _ = bench
    assert mod.VALU_PEAK_TLOPS == pytest.approx(256 * 64 * 2.4e9 / 1e12)
    assert 2 * mod.VALU_PEAK_TLOPS == pytest.approx(78.6, abs=0.05)
