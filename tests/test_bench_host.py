"""Host-side logic of the benchmark: the committed rocprofv3 summaries carry one
machine-readable traffic line each, in the format bench.py parses, naming source
files that exist; the multi-GPU request is refused with a message (one GPU is
measured)."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAT = re.compile(r'^PMC_TRAFFIC kernel="([^"]+)" bytes_per_launch=(\d+) src_sha256=(\w+) srcs=(\S+)')


def test_profile_traffic_lines():
    pdir = os.path.join(ROOT, "profiles")
    found = {}
    for fn in sorted(os.listdir(pdir)):
        with open(os.path.join(pdir, fn)) as fh:
            text = fh.read()
        assert "rocprofv3" in text, fn  # every summary names the command that made it
        for ln in text.splitlines():
            m = PAT.match(ln.strip())
            if m:
                found[m.group(1)] = int(m.group(2))
                for src in m.group(4).split(","):
                    assert os.path.exists(os.path.join(ROOT, src)), src
    for kernel in ("k_syrk_split_pair_partial", "k_cols_schurIDF16b", "k_kernel_colsIDF16bff"):
        assert kernel in found and found[kernel] > 10**8, kernel


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
