"""Writes md_paper_4096_digests.txt: SHA-256 digests of the oracle's output
frames for the full-size paper pipeline workload (Sec. 4.1, Gauss 5x5 ->
Thres -> Med 5-px, 4096 frames of 320x240, threshold 20, seed 28), one
digest per block of 64 consecutive frames.  Calls only the oracle and the
seeded input generator.

    python tests/golden/make_md_paper_digests.py
"""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import md_paper as omd          # noqa: E402
from workloads import paper_motion          # noqa: E402

SEED, N_FRAMES, THRESHOLD, BLOCK = 28, 4096, 20, 64
OUT = os.path.join(HERE, "md_paper_4096_digests.txt")


def block_digests(frames):
    out = omd.paper_motion_direct(frames, THRESHOLD)
    return [hashlib.sha256(out[b:b + BLOCK].tobytes()).hexdigest() for b in range(0, len(out), BLOCK)]


def main():
    w = paper_motion(seed=SEED, n_frames=N_FRAMES)
    with open(OUT, "w") as fh:
        fh.write("# Oracle output digests, paper motion-detection pipeline (Sec. 4.1),\n")
        fh.write(f"# seed {SEED}, {N_FRAMES} frames of 320x240, threshold {THRESHOLD};\n")
        fh.write(f"# SHA-256 of each block of {BLOCK} output frames (u8, row-major).\n")
        fh.write("# Written by make_md_paper_digests.py from the oracle only.\n")
        for k, d in enumerate(block_digests(w.frames)):
            fh.write(f"{k * BLOCK} {d}\n")


if __name__ == "__main__":
    main()
