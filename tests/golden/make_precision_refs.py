"""Write tests/golden/precision_refs.json: the exact sum S* and sum |x| (each
rounded once to double by the oracle's superaccumulator) of the 2^30-item
float32 columns that the benchmark's precision report uses.  Calls only the
input generator and the oracle; the benchmark reads the stored values (it
may not run the oracle outside its CPU-baseline leg), and
tests/test_precision_bound.py recomputes them.

    python tests/golden/make_precision_refs.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402
import oracle   # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_refs.json")
COLUMNS = [  # (name, distribution, seed): the benchmark's float32 column and the precision study's
    ("f32_uniform_seed4", "uniform", 4),
    ("f32_normal_outliers_seed11", "normal_outliers", 11),
]
N = 1 << 30


def compute(dist, seed, n=N):
    x = datagen.column(n, "f32", dist, seed=seed)
    return {"n": n, "dtype": "f32", "dist": dist, "seed": seed,
            "exact_sum": oracle.aggregate(x, "sum").f64, "abs_sum": oracle.aggregate(x, "abs_sum").f64}


def main():
    refs = {"about": "exact sum S* and sum|x| of seeded 2^30-item float32 columns, from the oracle "
                     "(written by make_precision_refs.py)",
            "columns": {name: compute(dist, seed) for name, dist, seed in COLUMNS}}
    with open(OUT, "w") as f:
        json.dump(refs, f, indent=1)
        f.write("\n")
    print(json.dumps(refs, indent=1))


if __name__ == "__main__":
    main()
