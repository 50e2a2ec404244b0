"""The oracle's parallel loops change no result: a bed stepped, coupled and
reacted on one thread and on several gives bit-identical pairs, forces,
states and sources (no GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_03908_amd import workloads as W


def _run(w, threads):
    O.set_threads(threads)
    try:
        ora = O.Oracle(w)
        out = {"pairs": ora.pairs()}
        out["F"], out["T"] = ora.forces()
        out["Fs"], out["Ts"] = ora.force_scale()
        ora.step(4)
        out.update({"c_" + k: v for k, v in ora.couple().items()})
        out.update({"r_" + k: np.asarray(v) for k, v in ora.react(1e-3, n_beds=len(w.beds)).items()})
        out.update({"s_" + k: v for k, v in ora.state().items()})
        return out
    finally:
        O.set_threads(1)


@pytest.mark.parametrize("case", ["cylinder", "beds"])
def test_results_independent_of_thread_count(case):
    if case == "cylinder":
        w = W.with_velocities(W.squeeze(W.cfg2(n=6000, seed=3), 0.97, 0), 3, vscale=0.03, wscale=20.0)
        w.params["mu_r"] = 2e-5
    else:
        w = W.with_velocities(W.squeeze(W.cfg5(n_beds=3, n_scale=0.03, seed=4), 0.97, 0), 4)
    one = _run(w, 1)
    many = _run(w, 4)
    assert len(one["pairs"]) > 100
    for k in one:
        assert np.array_equal(one[k], many[k]), k
