"""Quadrotor and integrator configuration values used by every workload.

The airframe numbers (mass 1.0 kg, arm 0.15 m, inertia diag(0.0025, 0.0025,
0.0045) kg m^2, rotor time constant 0.03 s, linear drag 0.1 N s/m, control step
0.02 s) are the benchmark configuration.  The constants the paper leaves open
(Sec. III-A, Eqs. 2-4 and the controller paragraph) take these readings:
yaw reaction ratio 0.016 m, per-rotor thrust limit 0.75 m g (thrust-to-weight 3),
body-rate gains diag(20, 20, 10) 1/s, gravity 9.81 m/s^2 along -z, no quadratic
drag term, one sub-step per control step, RK4 integration, CTBR control.
The position / velocity controllers (PS, LV) use position gains 4 1/s^2,
velocity gains 4 1/s, attitude gains (8, 8, 4) 1/s and a 45 degree tilt limit
(readings: the paper names the controllers but gives no law or gains).

Values are plain Python floats; callers cast them to float32 for the device.
"""

# Field order of the parameter block (mirrors the C struct ``vf_dyn_params``).
PARAM_FIELDS = (
    "dt", "n_sub", "integrator", "ctrl",
    "mass", "arm", "J", "tau_motor", "kappa_yaw", "f_max",
    "k_lin", "c_quad", "g", "k_rate",
    "k_pos", "k_vel", "k_att", "max_tilt",
)

INTEGRATOR_RK4 = 0
INTEGRATOR_EULER = 1
CTRL_CTBR = 0
CTRL_SRT = 1
CTRL_PS = 2
CTRL_LV = 3


def default_params(**overrides):
    """Return the benchmark airframe/integrator configuration as a dict."""
    g = 9.81
    mass = 1.0
    p = {
        "dt": 0.02,
        "n_sub": 1,
        "integrator": INTEGRATOR_RK4,
        "ctrl": CTRL_CTBR,
        "mass": mass,
        "arm": 0.15,
        "J": (0.0025, 0.0025, 0.0045),
        "tau_motor": 0.03,
        "kappa_yaw": 0.016,
        "f_max": 0.75 * mass * g,
        "k_lin": (0.1, 0.1, 0.1),
        "c_quad": (0.0, 0.0, 0.0),
        "g": g,
        "k_rate": (20.0, 20.0, 10.0),
        "k_pos": (4.0, 4.0, 4.0),
        "k_vel": (4.0, 4.0, 4.0),
        "k_att": (8.0, 8.0, 4.0),
        "max_tilt": 0.7853981633974483,
    }
    for k, v in overrides.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    return p


def device_params(p):
    """The parameter values the device receives: every real field rounded to float32 once (the C parameter
    block holds float32), as plain Python floats.  Comparing the FP64 oracle with the device on these
    values compares the arithmetic, with the same inputs on both sides."""
    import numpy as np
    out = {}
    for k, v in p.items():
        if isinstance(v, float):
            out[k] = float(np.float32(v))
        elif isinstance(v, tuple):
            out[k] = tuple(float(np.float32(x)) for x in v)
        else:
            out[k] = v
    return out
