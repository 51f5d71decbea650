"""Writes coexistence_pr.json: the critical temperature and the Maxwell
equal-area coexistence densities of the Peng-Robinson EOS (Eq. 56) with the
paper's a = 3/49, b = 2/21, R = 1, omega = 0.344 at T = 0.86 Tc (Sec. III.B).
Calls only the oracle."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main():
    cfg = dict(a=3.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344)
    tc = oracle.Tc(cfg["a"], cfg["b"], cfg["R"])
    rv, rl, ps = oracle.maxwell(cfg, 0.86 * tc)
    out = dict(cite="Eq. (56); a, b, R, omega and T_sat = 0.86 Tc of Sec. III.B",
               a=cfg["a"], b=cfg["b"], R=cfg["R"], omega=cfg["omega"],
               Tc=tc, T_over_Tc=0.86, rho_v=rv, rho_l=rl, p_sat=ps)
    with open(os.path.join(HERE, "coexistence_pr.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
