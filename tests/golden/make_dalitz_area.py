"""Writes dalitz_area.json: the area of the D+ -> h- h+ h+ Dalitz region (Sec. 4 kinematics) for the
pion and kaon final states, by adaptive quadrature of the oracle's s13 range over s12, and the share
of the bounding square [s_min, s_max]^2 that it covers.  Run from the repository root:
    python tests/golden/make_dalitz_area.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import Model  # noqa: E402
from oracle import kinematics as K  # noqa: E402

M_D, M_PI, M_K = 1.86966, 0.13957, 0.493677


def main():
    out = {"_source": "Area of the D+ -> h- h+ h+ Dalitz region (Sec. 4 kinematics; M = 1.86966, m_pi = 0.13957, "
                      "m_K = 0.493677 GeV): the integral over s12 of the s13 range, by adaptive quadrature at "
                      "1e-14 (written by make_dalitz_area.py). Box acceptance = area / (s_max - s_min)^2."}
    for name, m in (("pipipi", M_PI), ("kkk", M_K)):
        model = Model(M_D, m, m, m, 5.0, (0.0, 1.0), ())
        a = K.area(model)
        out[name] = round(a, 12)
        if name == "pipipi":
            out["pipipi_box_acceptance"] = round(a / (K.smax(model) - K.smin(model)) ** 2, 9)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dalitz_area.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=2)
        f.write("\n")
    print(out)


if __name__ == "__main__":
    main()
