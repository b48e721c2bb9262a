"""Grasp evaluation of the paper (Sec. IV-A controller, Sec. IV-B force sensing,
Sec. V simulation procedure: AutoGrasp, Lift, Shake) on the oracle scene.

Test infrastructure: a plain transcription of the procedure that drives
`oracle.ref.RefScene` step by step; only tests and the benchmark's CPU leg use it.

Readings (where the paper leaves a choice):
  * the controller's target for the next step is the gripper's current state plus
    phi(f) times the joint increment; for a two-finger gripper each finger is one joint
    whose increment is its closing velocity times h, and f is the magnitude of the
    contact force on that finger;
  * AutoGrasp stops when every finger's phi is zero, i.e. its force has reached f*
    (the paper stops at 1 N per finger: run with f* = 1 N for that), or after a cap;
  * Lift moves every finger along -gravity at a fixed speed for a number of steps;
    Shake displaces every finger by a(t) = A sin(2 pi f t) along one axis;
  * success: at the end some finger carries a nonzero contact force (the object is in
    the hand) and the ground carries none (the object does not touch the ground).
"""
import math

import numpy as np


def phi(f, k=20.0, f_star=0.5):
    """The force controller's gain (Sec. IV-A eq. 12): decays from 1 at f = 0 to 0 at the
    desired force f*, and stays 0 beyond it."""
    if f >= f_star:
        return 0.0
    return (math.exp(-k * f) - math.exp(-k * f_star)) / (1.0 - math.exp(-k * f_star))


def finger_layout(scene):
    """(affine index, DOF offset, closing velocity) of every driven affine body: the DOF
    vector holds the soft vertices, then the q of every non-fixed affine body in
    creation order."""
    nsv = sum(len(b.rest_pos) for b in scene.softs)
    out, off = [], 3 * nsv
    for i, b in enumerate(scene.affines):
        if b.mode == 1:                      # fixed: not in the DOF vector
            continue
        if b.mode == 2:
            out.append((i, off, np.asarray(b.target_vel, dtype=float)))
        off += 12
    return out


def run(R, scene, k=20.0, f_star=0.5, max_close_steps=200, lift_steps=100, lift_speed=0.1, shake_steps=0,
        shake_amplitude=0.0, shake_frequency=0.0, shake_axis=(1.0, 0.0, 0.0), object_body=0, ground_body=-1):
    """AutoGrasp, Lift, Shake on the oracle scene R; returns (result, trace) with trace
    rows [phase, |f_ground|, |f_finger| ...] measured before every step."""
    h = scene.params.dt
    g = np.asarray(scene.params.gravity, dtype=float)
    up = -g / np.linalg.norm(g) if np.linalg.norm(g) > 0 else np.array([0.0, 1.0, 0.0])
    fingers = finger_layout(scene)
    nsb = len(scene.softs)
    axis = np.asarray(shake_axis, dtype=float)
    phase, in_phase, n = 0, 0, 0
    close_steps = 0
    trace = []
    while True:
        y = R.get_state()[0]
        F = R.contact_forces(y)
        fmag = [float(np.linalg.norm(F[nsb + i])) for i, _, _ in fingers]
        fground = float(np.linalg.norm(F[ground_body])) if ground_body >= 0 else 0.0
        if phase == 0 and (all(phi(f, k, f_star) == 0.0 for f in fmag) or in_phase >= max_close_steps):
            close_steps = in_phase
            phase, in_phase = 1, 0
        if phase == 1 and in_phase >= lift_steps:
            phase, in_phase = 2, 0
        if phase == 2 and in_phase >= shake_steps:
            break
        trace.append([phase, fground] + fmag)
        for (i, off, vel), f in zip(fingers, fmag):
            q = y[off:off + 12].copy()
            if phase == 0:
                q[:3] += phi(f, k, f_star) * h * vel
            elif phase == 1:
                q[:3] += lift_speed * h * up
            else:
                a0 = shake_amplitude * math.sin(2.0 * math.pi * shake_frequency * in_phase * h)
                a1 = shake_amplitude * math.sin(2.0 * math.pi * shake_frequency * (in_phase + 1) * h)
                q[:3] += (a1 - a0) * axis
            R.set_drive_target(i, q)
        R.step(1)
        n += 1
        in_phase += 1
    fmax = max(fmag) if fmag else 0.0
    res = {"close_steps": close_steps, "total_steps": n, "success": int(fmax > 0.0 and fground == 0.0),
           "ground_force": fground, "finger_force_max": fmax, "n_fingers": len(fingers)}
    return res, np.array(trace).reshape(-1, 2 + len(fingers))
