"""Paper pin on the GPU: the HIP path replays the mesh histories of the
paper's adaptive runs (Section 5.2) and must reproduce every printed element
count (tests/golden/paper_element_counts.csv).  The 3D slab runs directly,
as a periodic cube of 16 identical level-4 layers."""
import pytest

import replay
from paper_2306_06744_amd import synth

pytestmark = pytest.mark.gpu

COUNTS = replay.paper_counts()


def replay_gpu(name):
    import paper_2306_06744_amd as lt
    run = replay.runs()[name]
    nodes = synth.gl_nodes01(run.p)
    t = lt.Tree.uniform(run.dim, run.d_min, run.d_max, depth=run.start_depth)
    f = None
    for k in [0] * run.warmup + list(range(run.cycles)):
        f = t.flag([run.centre(k)], 5.0, 6.0, nodes, run.lo, run.length, dist_axes=2,
                   periodic_dist=True, out=f if f is not None and f.numel() == t.size() else None)
        t.adapt(f)
        t.balance()
        f = None
    return t.size() // run.z_layers


@pytest.mark.parametrize("name", sorted(COUNTS))
def test_paper_element_count_gpu(name):
    print("replay", name, flush=True)
    got = replay_gpu(name)
    print(name, got, COUNTS[name], flush=True)
    assert got == COUNTS[name]
