"""Seeded synthetic inputs for the dense RGB-D-inertial tracking step.

This package only *generates* inputs: a procedural scene (three planes and
four spheres with a value-noise albedo), smooth camera trajectories, IMU
samples along them, and the workload configurations built from those pieces.
It holds none of the tracking method's arithmetic; both the CPU oracle and the
GPU path consume what it produces.  The paper's own datasets (a re-rendered
ICL-NUIM living room and a RealSense ZR300 + Vicon recording, Section VI) are
not available, and these generators stand in for them.
"""
from .scene import Scene, make_scene, render
from .trajectory import BSplineTrajectory, ConstantTwistTrajectory, make_spline_trajectory
from .imu_gen import ImuNoise, synth_imu
from . import configs

__all__ = [
    "Scene", "make_scene", "render",
    "BSplineTrajectory", "ConstantTwistTrajectory", "make_spline_trajectory",
    "ImuNoise", "synth_imu", "configs",
]
