#!/usr/bin/env python3
"""Writes large_leaf_blobs.txt: the oracle's serialized structures for key sets
whose buckets hold split nodes at leaf sizes 17-24.

The oracle needs from tens of seconds to a few minutes per set (leaves of 20-24
keys take m^m/m! ~ 10^8-10^9 trials each), too long to recompute in every GPU
test run, so the GPU parity tests compare with these stored bytes.  This script
calls only the oracle and the seeded input generators.

Shapes (leaf l, bucket b, keys n, input seed):
  l=20, b=160, n=320: about two buckets of 160 keys; a node of at most
      s*l = 160 keys splits into 8 parts of 20 (eight fields of 8 bits packed
      into one 64-bit counter).
  l=22, b=200, n=198: one bucket of 198 keys = 9 parts of 22, the only fanout
      that counts against 8 thresholds (s = 9 from l = 22 on).  Input seed
      3237 is one whose 9-way split succeeds early (index 581,094 against a
      mean of about 10^8 trials, which on one wavefront takes minutes).
  l=24, b=48, n=48: one bucket of 48 keys split into two leaves of 24.
  l=18, b=120, n=360: three buckets around 120 keys; lower-level nodes of up
      to 7 * 18 = 126 keys split into parts of 18 (packed counters).
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SHAPES = [(20, 160, 320, 2020), (22, 200, 198, 3237), (24, 48, 48, 2024), (18, 120, 360, 2018)]
OUT = os.path.join(HERE, "large_leaf_blobs.txt")


def one(shape):
    import oracle
    from paper_1910_06416_amd import inputs

    leaf, bucket, n, seed = shape
    keys = inputs.u64_keys(n, seed)
    blob = oracle.build(keys, leaf, bucket)
    return leaf, bucket, n, seed, blob.hex()


def main():
    with ProcessPoolExecutor(max_workers=len(SHAPES)) as ex:
        rows = list(ex.map(one, SHAPES))
    with open(OUT, "w") as f:
        f.write("# Oracle structures of inputs.u64_keys(n, seed) at leaf sizes 17-24 (written by\n")
        f.write("# make_large_leaf_blobs.py, which calls only the oracle).\n")
        f.write("# leaf bucket n seed blob_hex\n")
        for leaf, bucket, n, seed, hx in rows:
            f.write(f"{leaf} {bucket} {n} {seed} {hx}\n")
    print(OUT)


if __name__ == "__main__":
    main()
