"""The c2 and c3 workloads against the oracle value for value: every
1024-row tile the GPU delivers has the digest of the oracle's own tile, in
the default launch configuration (graph replays, lanes-per-row long rows)
and with the long rows on the segmented kernel: c2 and c3 in full (5.0e7
and 1.1e8 pairs, sequences up to 1,960 residues).  The digests were written
by tests/golden/make_oracle_digests.py, which runs only the oracle; a family
the file leaves out is skipped here."""
import hashlib
import os

import numpy as np
import pytest

from paper_1603_06958_amd import binding as B
from paper_1603_06958_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    """Digests per (family, row_begin, row_end), and the families left out."""
    path = os.path.join(GOLDEN, f"oracle_digests_{name}.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_oracle_digests.py {name})")
    head = open(path).readline()
    assert f"generator version {inputs.GENERATOR_VERSION}," in head
    out, skipped = {}, set()
    for line in open(path):
        if line.startswith("# families left out"):
            skipped = {int(x) for x in line.split(":", 1)[1].split() if x != "none"}
        if line.startswith("#"):
            continue
        f, r0, r1, n, h = line.split()
        out[(int(f), int(r0), int(r1))] = (int(n), h)
    return out, skipped


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["c2", "c3"])
@pytest.mark.parametrize("flags", [0, B.LONG_SEGMENTED | B.NO_GRAPH])
def test_every_value_equals_the_oracle(name, flags):
    want, skipped = load(name)
    b = getattr(inputs, name)()
    print(f"{name}: {len(want)} tiles, flags {flags:#x}, families left out {sorted(skipped)}", flush=True)
    got = {}

    def fn(t):
        if int(t.family) in skipped:
            return 0
        v = np.ascontiguousarray(B.tile_array(t), dtype="<i4")
        got[(int(t.family), int(t.row_begin), int(t.row_end))] = (v.size,
                                                                  hashlib.blake2b(v.tobytes(), digest_size=16).hexdigest())
        return 0

    with B.Plan.from_batch(b, tile_rows=1024, flags=flags) as p:
        p.run(fn)
    assert got.keys() == want.keys()
    bad = [key for key in want if got[key] != want[key]]
    assert not bad, f"{len(bad)} of {len(want)} tiles differ from the oracle, first {bad[0]}"
