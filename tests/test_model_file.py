"""The model-file format of the paper's model parser (section 5, table "Model
parser"): the printed predator-prey example parses to the Lotka-Volterra
network the benchmarks use, files round-trip exactly, and malformed files are
rejected with the line at fault."""
import os

import numpy as np
import pytest

from paper_2103_00405_amd import model_file as MF
from paper_2103_00405_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lotka_volterra_model.txt")


def _same_net(a, b):
    for f in ("react_ptr", "react_species", "react_sigma", "prod_ptr", "prod_species",
              "prod_mult"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.array_equal(a.c.view(np.uint64), b.c.view(np.uint64))
    assert (a.N, a.M) == (b.N, b.M)


def test_paper_example_is_lotka_volterra():
    m = MF.load(GOLDEN)
    assert m.net.names == ("A", "B")
    assert m.x0.tolist() == [1000, 1000]
    assert m.t_end == 2.0 and m.steps == 10000
    # A -> 2A (10), A + B -> 2B (0.01), B -> 0 (10): the benchmark network
    _same_net(m.net, W.lotka_volterra((10.0, 0.01, 10.0)))
    g = MF.sample_grid(m)
    assert len(g) == 10000 and g[0] == 0.0 and g[-1] == 2.0


def test_round_trip_exact():
    m = MF.load(GOLDEN)
    m2 = MF.parse(MF.dumps(m, comment="round trip"))
    _same_net(m.net, m2.net)
    assert np.array_equal(m.x0, m2.x0) and m.t_end == m2.t_end and m.steps == m2.steps
    rng = np.random.default_rng(11)
    for N, M in ((3, 7), (20, 60), (200, 900)):
        net = W.random_network(N, M, rng)
        net = net._replace(names=tuple("S%d" % j for j in range(N)))
        x0 = rng.integers(0, 500, size=N).astype(np.int32)
        m = MF.Model(net, x0, 0.125, 7)
        m2 = MF.parse(MF.dumps(m))
        _same_net(net, m2.net)
        assert np.array_equal(x0, m2.x0)


def test_duplicate_species_add_up_and_comments():
    m = MF.parse("""
        // dimerisation
        # init
        A = 10   // monomer
        B = 0
        # reactions
        1 A 1 A --> 1 B : 0.5
        1 B --> 2 A : 1e-1
        # end
        time = 1.5
        steps = 3
    """)
    net = m.net
    assert net.react_sigma.tolist() == [2, 1] and net.prod_mult.tolist() == [1, 2]
    _same_net(net, W.dimerisation(0.5, 0.1)._replace(names=("A", "B")))


@pytest.mark.parametrize("text,msg", [
    ("# reactions\n1 A --> NULL : 1\n# end\ntime = 1\nsteps = 2\n", "order"),
    ("# init\nA = 1\n# reactions\n1 C --> NULL : 1\n# end\ntime = 1\nsteps = 2\n", "not declared"),
    ("# init\nA = 1\n# reactions\n2 A 1 A --> NULL : 1\n# end\ntime = 1\nsteps = 2\n", "more than 2"),
    ("# init\nA = 1\n# reactions\n1 A --> NULL : -1\n# end\ntime = 1\nsteps = 2\n", ">= 0"),
    ("# init\nA = 1\n# reactions\n1 A --> NULL : x\n# end\ntime = 1\nsteps = 2\n", "not a number"),
    ("# init\nA = 1\n# reactions\n1 A -> NULL : 1\n# end\ntime = 1\nsteps = 2\n", "expected"),
    ("# init\nA = 1\n# reactions\n1 A --> NULL : 1\n# end\ntime = 1\n", "steps"),
    ("# init\nA = -1\n# reactions\n1 A --> NULL : 1\n# end\ntime = 1\nsteps = 2\n", "count"),
    ("# init\nA = 1\nA = 2\n# reactions\n1 A --> NULL : 1\n# end\ntime = 1\nsteps = 2\n", "twice"),
    ("# init\nA = 1\n# reactions\n0 A --> NULL : 1\n# end\ntime = 1\nsteps = 2\n", "positive"),
    ("# init\nA = 1\n# reactions\n1 A --> NULL 1 A : 1\n# end\ntime = 1\nsteps = 2\n", "NULL"),
    ("# init\nA = 1\n# reactions\n1 A --> NULL : 1\n# end\ntime = 1\nsteps = 2\ndt = 3\n", "unknown"),
])
def test_rejects_malformed(text, msg):
    with pytest.raises(MF.ModelFileError, match=msg):
        MF.parse(text)


def test_oracle_runs_the_parsed_model():
    """The parsed example drives the CPU oracle like the catalogue network."""
    import oracle
    m = MF.load(GOLDEN)
    a = oracle.simulate(m.net, m.x0, 0.05, [0.05], 3, 4)
    b = oracle.simulate(W.lotka_volterra((10.0, 0.01, 10.0)), m.x0, 0.05, [0.05], 3, 4)
    assert np.array_equal(a["n"], b["n"]) and np.array_equal(a["samples"], b["samples"])


@pytest.mark.gpu
def test_gpu_runs_the_parsed_model_bit_exact():
    """The paper's example end to end on the GPU with its own grid (10000
    output points over t in [0, 2]), against the oracle."""
    import oracle
    import torch
    from paper_2103_00405_amd import api
    m = MF.load(GOLDEN)
    grid = MF.sample_grid(m)
    R = 48
    g = api.simulate(api.Network(m.net), m.x0, m.t_end, grid, R, seed=5, with_hash=True)
    torch.cuda.synchronize()
    ref = oracle.simulate(m.net, m.x0, m.t_end, grid, 5, R)
    assert np.array_equal(g["samples"].cpu().numpy(), ref["samples"])
    assert np.array_equal(g["n"].cpu().numpy().view(np.uint32), ref["n"])
    assert np.array_equal(g["T"].cpu().numpy().view(np.uint64), ref["T"].view(np.uint64))
    assert np.array_equal(g["seq_hash"].cpu().numpy().view(np.uint64), ref["seq_hash"])
