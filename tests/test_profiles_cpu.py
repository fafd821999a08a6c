"""The committed rocprofv3 counter summary of the headline GEMM was taken on
the current kernel sources: bench.py reports its traffic and MFMA utilisation
only for a summary line whose source hash matches, so a code change to the
GEMM kernel's sources without a new profile would leave them unreported."""
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_for_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_profile_matches_kernel_sources():
    b = _bench()
    h = b.source_hash()
    lines = [json.loads(l) for l in open(os.path.join(ROOT, "profiles", "bf16_gemm_4096_counters.txt"))
             if l.strip() and not l.startswith("#")]
    assert lines
    assert all(l["source_hash"] == h for l in lines), (h, {l["source_hash"] for l in lines})
    # every configuration the headline search can pick among is covered
    cfgs = {tuple(l["config"]) for l in lines}
    want = {(256, 256, 64, wm, wn, 1, gm, x, 2, 0, mf) for wm, wn in ((2, 4), (4, 2)) for gm in (1, 8)
            for x in (0, 1) for mf in (0, 32)}
    assert want <= cfgs, want - cfgs


def test_source_hash_ignores_comments(tmp_path):
    """A comment edit keeps the hash; a code edit changes it."""
    import shutil
    b = _bench()
    h = b.source_hash()
    csrc = tmp_path / "paper_2307_16080_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in b.KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2307_16080_amd", "csrc", name), csrc / name)
    b.ROOT = str(tmp_path)
    assert b.source_hash() == h
    k = csrc / "kernels.hpp"
    k.write_text(k.read_text() + "\n// a comment\n/* and a\n   block comment */\n")
    assert b.source_hash() == h
    k.write_text(k.read_text() + "\nstatic const int probe_value = 1;\n")
    assert b.source_hash() != h
