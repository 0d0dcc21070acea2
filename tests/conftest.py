import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run through the GPU runner)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def rgbd_small():
    import synth
    return synth.make("rgbd_small")


@pytest.fixture(scope="session")
def rgbd_small_clean():
    import synth
    return synth.make("rgbd_small", noise=False)


@pytest.fixture(scope="session")
def lidar_mini():
    """Two 48x768 spherical keyframes 6.7 m apart on the LiDAR loop (noisy)."""
    import synth
    full = synth.make("lidar128", kfs=[0, 1, 2], H=48, W=768)
    return full.subset([0, 1, 2])


@pytest.fixture(scope="session")
def lidar_mini_clean():
    import synth
    full = synth.make("lidar128", kfs=[0, 1, 2], H=48, W=768, noise=False)
    return full.subset([0, 1, 2])


JOINT_KFS = [0, 1, 2, 200, 201, 202, 203, 204]   # 3 LiDAR keyframes and 5 camera keyframes, 0-30 m


@pytest.fixture(scope="session")
def joint_mini():
    """A 30 m stretch of the joint rig: 32x256 LiDAR and 60x80 camera keyframes with sensor
    offsets; all four source/target model combinations occur among the 54 pairs."""
    import synth
    full = synth.make("joint", H_l=32, W_l=256, H_c=60, W_c=80, kfs=JOINT_KFS)
    return full.subset(JOINT_KFS)


@pytest.fixture(scope="session")
def joint_mini_clean():
    import synth
    full = synth.make("joint", H_l=32, W_l=256, H_c=60, W_c=80, kfs=JOINT_KFS, noise=False)
    return full.subset(JOINT_KFS)


def rot_angle_deg(Ra, Rb):
    c = (np.trace(Ra.T @ Rb) - 1.0) / 2.0
    return float(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))
