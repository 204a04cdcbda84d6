"""bench.py's command line: every documented workload reaches its runner, an unknown one
and more than one GPU are refused (host logic only; the runners are replaced by stubs)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


@pytest.mark.parametrize("workload,runner", [("c3", "run_c3"), ("c5", "run_c5"), ("sigma", "run_sigma"),
                                             ("real", "run_real"), ("eps", "run_eps")])
def test_each_workload_reaches_its_runner(workload, runner, monkeypatch):
    seen = []
    for name in ("run_c3", "run_c5", "run_sigma", "run_real", "run_eps"):
        monkeypatch.setattr(bench, name, lambda args, name=name: seen.append(name))
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", workload])
    bench.main()
    assert seen == [runner]


def test_unknown_workload_and_several_gpus_are_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "c9"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert "unknown workload" in str(e.value)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "8"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2 and "one GPU" in capsys.readouterr().err


def test_eps_roofline_counts_the_rank_updates():
    # NG = 128: two 64-wide block columns, each updating the 64 x 64 entries outside its rows
    # and columns with 64 complex multiply-adds (8 flops) per entry; two frequencies, 1 ms
    r = bench.roofline_eps({"eps_rank_update": {"ms_per_step": 1.0}}, 128, 2)
    flops = 2 * 2 * 8 * 64 * 64 * 64
    assert r["achieved"] == pytest.approx(flops / 1e-3 / 1e12)
    assert r["peak"] == 78.6 and r["frac"] == pytest.approx(r["achieved"] / 78.6)
    # a ragged last block: NG = 100 has blocks of 64 and 36
    r = bench.roofline_eps({"eps_rank_update": {"ms_per_step": 1.0}}, 100, 1)
    assert r["achieved"] == pytest.approx(8 * (36 * 36 * 64 + 64 * 64 * 36) / 1e-3 / 1e12)
    assert bench.roofline_eps({}, 100, 1) is None
