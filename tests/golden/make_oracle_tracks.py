"""Write the oracle's track set for the first event of the one-vertex,
40-track recipe (seed 1) to ``tiny_event0_tracks.txt``.

The stored file anchors the oracle against accidental change: any later edit
of its arithmetic that alters this output must be justified by the passage
of the paper it follows.  Calls only the oracle and the input generator.

    python tests/golden/make_oracle_tracks.py
"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2207_03936_amd import synth  # noqa: E402


def main():
    b = synth.make_batch("tiny", 1)
    eto, tho, th = oracle.reconstruct(b)
    with open(os.path.join(HERE, "tiny_event0_tracks.txt"), "w") as f:
        f.write("# oracle tracks of event 0 of the one-vertex 40-track recipe (seed 1),\n")
        f.write("# default tolerances; one track per line, event-local hit ids in traversal order\n")
        for t in range(int(eto[1])):
            f.write(" ".join(str(int(h)) for h in th[tho[t]:tho[t + 1]]) + "\n")


if __name__ == "__main__":
    main()
