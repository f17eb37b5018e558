"""Graph replay (pond_set_graph): the captured two-step sequence gives bitwise the same
results as launching every kernel, over several replays with the program's own work and
synchronizations between them, across odd step counts (the parity changes, the graph is
captured again), a change of t_end, and with the learned seed."""
import numpy as np
import pytest

from paper_2203_05477_amd import workloads as W

pytestmark = pytest.mark.gpu


def _same(a, b):
    # a tube that failed holds the same invalid values on both sides
    return all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


def _state(g):
    return g.conserved(), g.face_frames(), g.time()


@pytest.mark.parametrize("case", ["dmr_fp64", "dmr_mixed", "tubes_mixed", "dmr_eq_mixed", "tubes_sl_fp64"])
def test_graph_replay_matches_eager(case):
    from paper_2203_05477_amd import pond

    if case.startswith("dmr"):
        cfg, f = W.double_mach(96, 24, tol=1e-13 if case.endswith("fp64") else 1e-5)
    else:
        cfg, f = W.tube_batch(n_tubes=64, len_lo=50, len_hi=300, tol=1e-5, rho_decades=1.0,
                              p_decades=1.0, mach=1.0)
    if "_eq_" in case:
        cfg["regularization"] = "eq"
    if "_sl_" in case:
        cfg["scheme"] = "sl"
    prec = "fp64" if case.endswith("fp64") else "mixed"
    eager = pond.Context(cfg, f, precision=prec)
    graph = pond.Context(cfg, f, precision=prec)
    graph.set_graph(True)
    print("case", case, flush=True)
    for n in (6, 6, 5, 4, 7, 2):
        se = eager.step(n, check=False)
        sg = graph.step(n, check=False)
        assert _same(_state(eager), _state(graph)), n
        assert se["iters_total"] == sg["iters_total"] and se["cell_updates"] == sg["cell_updates"]
    # a t_end inside the next steps: the graph is captured again with the clipped last step
    t = eager.time().max()
    eager.step(10, t_end=t * 1.02, check=False)
    graph.step(10, t_end=t * 1.02, check=False)
    assert _same(_state(eager), _state(graph))


def test_graph_replay_with_learned_seed():
    import torch

    from paper_2203_05477_amd import learned_seed as LS
    from paper_2203_05477_amd import pond

    cfg, f = W.double_mach(96, 24, tol=1e-5)
    data = LS.harvest(cfg, f, steps=40, precision="mixed", hard_iters=2)
    net, _, _ = LS.train([data], epochs=3, batch=1024, lr=2e-3)
    eager = pond.Context(cfg, f, precision="mixed", seed="mlp")
    graph = pond.Context(cfg, f, precision="mixed", seed="mlp")
    eager.load_mlp(net, hard_iters=2)
    graph.load_mlp(net, hard_iters=2)
    graph.set_graph(True)
    for n in (4, 4, 3, 6):
        eager.step(n)
        graph.step(n)
        assert _same(_state(eager), _state(graph)), n
    torch.cuda.synchronize()
