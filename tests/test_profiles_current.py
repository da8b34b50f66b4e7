"""The committed rocprofv3 summaries describe the current step: each carries
the digest of the step kernel and layout source it was taken on, and
bench.py reports the measured traffic only when that digest, the timed
kernel instance and the workload's fluid count all match.  A change to the
step's source needs the profiles taken again."""
import glob
import json
import os

import numpy as np

import bench

PROFILES = os.path.join(bench.ROOT, "profiles")


def test_traffic_profiles_match_the_current_step_and_workload():
    solid = bench.workload()[0]
    n_fluid = int(np.count_nonzero(solid == 0))
    digest = bench.kernel_hash()
    for prec, kernel in (("fp32", "step_kernel<float,64,16,MODE_STEP>"),
                         ("fp16s", "step_kernel<__half,64,16,MODE_STEP>")):
        t = json.load(open(os.path.join(PROFILES, f"traffic_step_{prec}_packed_spheres_256.json")))
        assert t["kernel_and_layout_source_sha256_16"] == digest, f"{prec} traffic profile is stale"
        assert t["kernel"] == kernel
        assert f"{n_fluid} fluid sites" in t["workload"]
        assert t["hbm_bytes_per_launch"] == t["hbm_read_bytes_per_launch"] + t["hbm_write_bytes_per_launch"]
    assert bench.traffic_for("step_kernel<float,64,16,MODE_STEP>", n_fluid) is not None


def test_summaries_name_the_current_source():
    digest = bench.kernel_hash()
    for path in glob.glob(os.path.join(PROFILES, "*.md")):
        assert digest in open(path).read(), f"{os.path.basename(path)} was taken on another source"
