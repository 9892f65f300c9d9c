"""Host-side checks of bench.py (no GPU): the one-GPU refusal, the byte models
it reports against, and the stored traffic summaries it reads."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_byte_models_are_the_per_pass_figures():
    # k / omega sweeps 2 x 144 B/cell and momentum sweeps 224 B/cell for n_s = 2,
    # split over 4 one-colour launches; the other passes one launch each
    assert bench.ALGO_BYTES["scalar_sweep"] * 4 == 144
    assert bench.ALGO_BYTES["mom_sweep"] * 4 == 224
    # momentum assembly: the 97 B/cell of the state it reads and writes plus the
    # three explicit terms; their pass reads u, v, w, nu_t (and p, k for the
    # iteration means) and writes the terms
    assert bench.ALGO_BYTES["mom_assemble"] == 97 + 24
    assert bench.ALGO_BYTES["mom_explicit"] == 48 + 24
    assert bench.ALGO_BYTES["scalar_assemble"] * 2 == 160
    assert bench.ALGO_BYTES["p_apply"] == 25
    # the fine-level pressure passes of one CG iteration with two sweeps per side
    # (pre-smoothing pass, one more red-black sweep, restriction, four post half
    # sweeps, apply with direction update, vector update): 302 B/cell
    b = bench.ALGO_BYTES
    assert b["p_presmooth"] + 2 * b["p_smooth"] + b["p_restrict"] + 4 * b["p_smooth"] + b["p_apply_dir"] + \
        b["p_axpy"] == 302
    for cls in bench.ALGO_BYTES:
        assert bench.KERNEL[cls].startswith("k_") and bench.KERNEL[cls] in bench.KERNEL_SOURCES
        assert bench.KERNEL_MIXED[cls] in bench.KERNEL_SOURCES


def test_stored_traffic_summaries_parse():
    # every committed traffic summary names its kernel's source hash and a byte count;
    # bench.py reports it only while that hash equals the current sources' hash
    prof = os.path.join(ROOT, "profiles")
    names = [n for n in os.listdir(prof) if n.startswith("traffic_") and n.endswith(".md")]
    assert names
    for n in names:
        text = open(os.path.join(prof, n)).read()
        assert "source_sha256" in text and "traffic_bytes_per_launch" in text, n
        kernel = n[len("traffic_"):].split("_ahmed")[0]
        assert kernel in bench.KERNEL_SOURCES, n
        h = bench.kernel_source_hash(kernel)
        t = bench.stored_traffic(kernel, "ahmed_256x96x96_sst_fp64")
        assert (t is None) == (h not in text), n
