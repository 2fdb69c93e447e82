"""The library's environment switches, on the CPU: HDC_LOG=1 prints one line
per dispatch decision on stderr; HDC_TUNE=0 keeps every tuning cache from
being read at start-up (the built-in defaults apply), HDC_TUNE_CACHE names the
cache otherwise.  Each case runs in a fresh process, since the switches are
read once."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# a map class line that differs from the built-in defaults in every field
CACHE_LINE = "0 0 0 3 128 2 16 8192 64 4 1\n"
TUNED = {"block": 128, "unroll": 2, "grid_mult": 16, "chunk": 8192, "small_seg": 64, "seg_per_wave": 4, "passes": 1}


def run(code, **env):
    e = dict(os.environ)
    for k in ("HDC_LOG", "HDC_TUNE", "HDC_TUNE_CACHE"):
        e.pop(k, None)
    e.update({k: v for k, v in env.items() if v is not None})
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=e, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stderr
    return p


GET_MAP = ("import json, paper_2309_03912_amd as hdc; "
           "print(json.dumps(hdc.get_tuning(hdc.OP_MAP, hdc.F32, hdc.ACC_PLAIN, 3)))")


def tuning_of(**env):
    return json.loads(run(GET_MAP, **env).stdout.strip().splitlines()[-1])


def test_tune_cache_read_unless_tune_0(tmp_path):
    cache = tmp_path / "cache.txt"
    cache.write_text("# test cache\n" + CACHE_LINE)
    assert tuning_of(HDC_TUNE_CACHE=str(cache)) == TUNED
    assert tuning_of(HDC_TUNE_CACHE=str(cache), HDC_TUNE="1") == TUNED
    defaults = tuning_of(HDC_TUNE_CACHE=str(cache), HDC_TUNE="0")
    assert defaults != TUNED
    assert defaults["passes"] == 2  # the built-in default


def test_tune_0_skips_the_shipped_cache():
    shipped = tuning_of()
    defaults = tuning_of(HDC_TUNE="0")
    # the shipped cache tunes the f32 map class at the largest bucket
    assert shipped != defaults
    line = [l.split() for l in open(os.path.join(ROOT, "paper_2309_03912_amd", "tuning_gfx950.txt"))
            if l.strip() and not l.startswith("#") and l.split()[:4] == ["0", "0", "0", "3"]]
    assert line and shipped["block"] == int(line[0][4]) and shipped["unroll"] == int(line[0][5])


def test_log_lines(tmp_path):
    code = ("import torch, paper_2309_03912_amd as hdc; "
            "x = torch.linspace(-1, 1, 1000); "
            "hdc.host_map(x, hdc.affine(2.5, 0.5), threads=2); "
            "hdc.host_transform_reduce(x, hdc.identity(), 'compensated', threads=3)")
    quiet = run(code)
    assert "hdc:" not in quiet.stderr
    off = run(code, HDC_LOG="0")
    assert "hdc:" not in off.stderr
    on = run(code, HDC_LOG="1")
    lines = [l for l in on.stderr.splitlines() if l.startswith("hdc: ")]
    assert any(l.startswith("hdc: host_map dtype=f32 n=1000 threads=2") for l in lines), on.stderr
    assert any(l.startswith("hdc: host_transform_reduce dtype=f32 acc=compensated n=1000 threads=3")
               for l in lines), on.stderr


def test_log_reports_the_cache_decision(tmp_path):
    cache = tmp_path / "cache.txt"
    cache.write_text(CACHE_LINE)
    read = run(GET_MAP, HDC_LOG="1", HDC_TUNE_CACHE=str(cache))
    assert f"hdc: tuning cache {cache} read at start-up: " in read.stderr
    skipped = run(GET_MAP, HDC_LOG="1", HDC_TUNE_CACHE=str(cache), HDC_TUNE="0")
    assert f"hdc: HDC_TUNE=0: tuning cache {cache} not read, built-in defaults" in skipped.stderr
