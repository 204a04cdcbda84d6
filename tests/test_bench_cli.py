"""bench.py's command line: every documented workload reaches its runner, an unknown one
and more than one GPU are refused (host logic only; the runners are replaced by stubs)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


@pytest.mark.parametrize("workload,runner", [("c3", "run_c3"), ("c5", "run_c5"), ("sigma", "run_sigma"),
                                             ("real", "run_real")])
def test_each_workload_reaches_its_runner(workload, runner, monkeypatch):
    seen = []
    for name in ("run_c3", "run_c5", "run_sigma", "run_real"):
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
