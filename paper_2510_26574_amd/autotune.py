"""Block-size autotuning for the batched form, with a JSON cache (host side).

Jobs fall into classes by rank budget r, dimension d and log2 of N; one job
per class is timed with each candidate block size through the library's
rpc_autotune_block, and the fastest b is cached under the class key so
later runs reuse it.  The chosen b is part of the job (it changes which
pivots are drawn), so it is recorded with the results.
"""
import json
import math
import os

BLOCKS = (16, 32, 64, 128)


def job_class(N, d, r):
    return f"r{int(r)}_d{int(d)}_n{2 ** int(round(math.log2(max(int(N), 1))))}"


def candidates(r):
    """Block sizes that divide r and leave at least two rounds."""
    return [b for b in BLOCKS if r % b == 0 and b <= r // 2] or [max(1, r // 2)]


def load_cache(path):
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def save_cache(path, cache):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(problems, make_job, cache_path=None, reps=1, tuner=None):
    """Block size per problem.

    problems: list of (N, d, r); make_job(i, b) builds a job for problem i
    with block size b (only called for one representative per class).
    Returns (list of b, cache dict).  `tuner(job, cands, reps) -> (b, ms)`
    defaults to the library's rpc_autotune_block.
    """
    if tuner is None:
        from . import autotune_block as tuner
    cache = load_cache(cache_path)
    out = []
    for i, (N, d, r) in enumerate(problems):
        key = job_class(N, d, r)
        if key not in cache:
            cands = candidates(r)
            best, ms = tuner(make_job(i, cands[0]), cands, reps)
            cache[key] = {"b": int(best), "ms": {str(k): float(v) for k, v in ms.items()}}
            save_cache(cache_path, cache)
        out.append(int(cache[key]["b"]))
    return out, cache
