"""One HIP runtime per process: with PyTorch installed, libseraph binds to the
HIP runtime torch ships, so torch's streams and device memory can be handed to
the library, and importing torch after the library loads no second copy."""
import os

import pytest


def loaded(prefix):
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 6 and os.path.basename(parts[5]).startswith(prefix):
                paths.add(os.path.realpath(parts[5]))
    return paths


def test_single_hip_runtime_with_torch():
    import paper_1806_00762_amd as sr
    rt = sr.torch_hip_runtime()
    if rt is None:
        pytest.skip("torch brings no HIP runtime here")
    sr.lib()
    import torch  # noqa: F401  (loads torch's HIP libraries)
    import torch.cuda  # noqa: F401
    hip = loaded("libamdhip64.so")
    assert hip == {os.path.realpath(rt)}, f"HIP runtimes in this process: {sorted(hip)}"
    hsa = loaded("libhsa-runtime64.so")
    assert len(hsa) == 1, f"HSA runtimes in this process: {sorted(hsa)}"
