"""Writes three_level_model.json: the GW+C satellite series of the paper's
three-level core-hole model (section "Assessing the validity of GW+C for a
shake-up process in a minimal model", Fig. model_system).

The paper fixes the result in closed form: one excitation weight
gamma = rho^2 / Omega^2, satellites at eps_c^QP - k Omega, intensities in a
Poisson distribution (weight of order k: exp(-gamma) gamma^k / k!).  The two
coupling ratios rho/Omega = 0.5 and 1.0 are the ones shown in the figure.
Only `math` is used; no code of this repository is called.
"""
import json
import math
import os

cases = []
for ratio in (0.5, 1.0):
    g = ratio * ratio
    cases.append({
        "rho_over_Omega": ratio,
        "gamma": g,
        "poisson_weights": [math.exp(-g) * g ** k / math.factorial(k) for k in range(6)],
    })
out = {
    "citation": "three-level core-hole model: gamma = rho^2/Omega^2, satellites at "
                "eps^QP - k Omega with Poisson intensities; rho/Omega = 0.5 and 1.0 "
                "as in Fig. model_system",
    "cases": cases,
}
path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "three_level_model.json")
with open(path, "w") as f:
    json.dump(out, f, indent=1)
