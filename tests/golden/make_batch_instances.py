"""Writes batch_instances_4096.json: the frozen table of the batched
workload (workloads.batch_instances), so a change in the sampler or in
numpy's stream is caught by tests/test_workloads.py."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402

n, d, s = workloads.batch_instances()
with open(os.path.join(HERE, "batch_instances_4096.json"), "w") as f:
    json.dump({"sampler": "workloads.batch_instances(count=4096, seed=0x5EED)",
               "n": [int(x) for x in n], "d": [int(x) for x in d], "seed": [int(x) for x in s]}, f)
