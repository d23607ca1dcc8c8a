"""The oracle's derived joint parameters at the operating point the paper prints (the table
of physical defaults in Sec. "Parameter Provenance", stored with the citation in
tests/golden/paper_defaults.json): a trunk
segment of the default radius, density, Young's modulus and modulus of rupture gets
Kp = (pi/4) E r^4 / l (Eq. beam), M_max = sigma_r pi r^3 / 4 (Eq. break: modulus of rupture
times the section modulus of a solid circular section) and, in the stiffness-proportional
damping mode, Kd = c_d Kp.  CPU only."""
import json
import math
import os

from orchard_inputs import assemble, chain_tree, step_constants
from oracle.oracle import Oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_defaults.json")


def test_trunk_segment_at_the_paper_defaults():
    g = {k: v["value"] for k, v in json.load(open(GOLDEN))["values"].items()}
    E, sr, rho, cd, r = (g["youngs_modulus_pa"], g["modulus_of_rupture_pa"], g["wood_density_kg_m3"],
                         g["damping_cd_s"], g["trunk_radius_m"])
    for length in (0.3, 0.6):
        t = chain_tree(1, length=length, radius=r, youngs=E, mor=sr, density=rho)
        d = Oracle(assemble([t]), step_constants(damping_cd=cd)).derived()
        kp = math.pi / 4 * E * r ** 4 / length
        mmax = sr * math.pi * r ** 3 / 4
        assert abs(d["kp"][0] - kp) <= 1e-12 * kp
        assert abs(d["mmax"][0] - mmax) <= 1e-12 * mmax
        assert abs(d["kd"][0] - cd * kp) <= 1e-12 * cd * kp
        # the joint breaks once it bends past M_max / Kp (0.061 rad for a 0.3 m segment)
        assert abs(d["mmax"][0] / d["kp"][0] - sr * length / (E * r)) <= 1e-12
