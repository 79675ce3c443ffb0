"""The benchmark's command line on the CPU: a GPU count other than one is
refused with a message and exit status 2 before anything touches a GPU."""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def test_more_than_one_gpu_is_refused(capsys):
    import bench
    assert bench.main(["--gpus", "2"]) == 2
    line = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
