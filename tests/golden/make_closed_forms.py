"""Writes closed_forms.json: closed-form values used as pins of the oracle.

Nothing here calls any implementation of the method; every value is a formula
evaluated with the math module.
  uniaxial_isochoric: F = diag(l, l^-1/2, l^-1/2), J = 1, I1 = l^2 + 2/l.
      neo-Hookean (mu_s, Psi = mu_s/2 (I1bar-3) + ...):
          P11 = (2 mu_s / 3)(l - l^-2),  P22 = (mu_s / 3)(l^-1/2 - l^5/2)
      Holzapfel-Ogden (a, b, a_f, b_f) with e_f = e_x, I4f = l^2:
          P11 = a exp(b (I1 - 3)) (2/3)(l - l^-2) + 2 a_f (l^2 - 1) exp(b_f (l^2-1)^2) l
  shell_net_pressure_force: the endocardial surface of the generated shell is
      open at the base (regular 224-gon, radius 0.21) and at the apex hole
      (regular 224-gon, radius 2h at h = 1/128); the net follower load per unit
      pressure is the difference of the polygon areas (1/2) m r^2 sin(2 pi / m).
  taylor_green_stokes_factor: per-step amplitude factor of the Taylor-Green
      mode under the Helmholtz step, 1 / (1 + (dt mu / rho) (8 / h^2) sin^2(pi h)).
"""
import json
import math
import os

lam, mu = 1.1, 10.0
a, b, af, bf = 0.5, 5.0, 1.5, 8.0
I1 = lam ** 2 + 2 / lam
out = {
    "uniaxial_isochoric": {
        "lambda": lam, "mu_s": mu,
        "nh_P11": 2 * mu / 3 * (lam - lam ** -2),
        "nh_P22": mu / 3 * (lam ** -0.5 - lam ** 2.5),
        "ho_params": [a, b, af, bf],
        "ho_P11": a * math.exp(b * (I1 - 3)) * 2 / 3 * (lam - lam ** -2)
        + 2 * af * (lam ** 2 - 1) * math.exp(bf * (lam ** 2 - 1) ** 2) * lam,
    },
    "shell_net_pressure_force": {
        "n_theta": 224, "r_base": 0.21, "r_apex": 2.0 / 128,
        "Fx_per_unit_p": 0.5 * 224 * (0.21 ** 2 - (2.0 / 128) ** 2) * math.sin(2 * math.pi / 224),
    },
    "taylor_green_stokes_factor": {
        "n": 32, "dt": 1e-3, "mu": 0.01, "rho": 1.0,
        "factor": 1.0 / (1.0 + 1e-3 * 0.01 * (8 * 32 ** 2) * math.sin(math.pi / 32) ** 2),
        "continuum": math.exp(-8 * math.pi ** 2 * 0.01 * 1e-3),
    },
}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json"), "w") as fh:
    json.dump(out, fh, indent=1)
