"""Writes robustness_oracle.txt: detection outcomes of the Section 5 scenes (targets and
clutter under AWGN and epsilon-contaminated Gaussian noise, noise-free reference) on the
FP64 oracle's surfaces of Eq. (12a), Eq. (12b) and the ordinary Eq. (11).

Calls only ``oracle`` (and the seeded generators of ``synth``). Run from the repository
root: ``python tests/golden/make_robustness.py``.
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "robustness_oracle.txt")
SURFACES = ("eq12a", "eq12b", "eq11")


def oracle_surfaces(scene: str, noise: str):
    import oracle
    import synth

    n, tau0, n_tau, p0, n_dop = synth.ROBUST_WINDOW
    s, r = synth.robustness_pair(scene, noise, n)
    return {
        "eq12a": oracle.caf(s, r, tau0, n_tau, p0, n_dop)[0],
        "eq12b": oracle.caf12b(s, r, tau0, n_tau, p0, n_dop)[0],
        "eq11": oracle.caf11(s, r, tau0, n_tau, p0, n_dop),
    }


def outcomes(scene: str, noise: str):
    import synth

    objs = synth.scene_objects(scene, synth.ROBUST_WINDOW[3])
    return {k: synth.object_margin(v, objs) for k, v in oracle_surfaces(scene, noise).items()}


def rows():
    import synth

    for scene in synth.ROBUST_SCENES:
        for noise in synth.ROBUST_NOISES:
            yield scene, noise, outcomes(scene, noise)


def format_row(scene, noise, surf, m) -> str:
    objs = " ".join("%.4f" % v for v in m["object_db"])
    return "%s | %s | %s | %d/%d | %.4f | %s" % (scene, noise, surf, m["detected"], m["objects"],
                                                m["margin_db"], objs)


def parse(path: str = OUT):
    """{(scene, noise, surface): (detected, objects, margin_db, [object_db])}"""
    out = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            scene, noise, surf, det, margin, objs = [t.strip() for t in line.split("|")]
            d, o = det.split("/")
            out[(scene, noise, surf)] = (int(d), int(o), float(margin), [float(v) for v in objs.split()])
    return out


def main():
    import synth

    n, tau0, n_tau, p0, n_dop = synth.ROBUST_WINDOW
    lines = [
        "# Detection outcomes on the FP64 oracle's surfaces (written by make_robustness.py,",
        "# which calls only the oracle). Scenes: Section 5 (targets and clutter under AWGN and",
        "# epsilon-contaminated Gaussian noise, reference noise free), N = %d, delays %d..%d," % (n, tau0, tau0 + n_tau - 1),
        "# Doppler bins %d..%d. Columns: scene | noise | surface (eq12a: Eq. (12a), eq12b:" % (p0, p0 + n_dop - 1),
        "# Eq. (12b), eq11: the ordinary Eq. (11)) | detected/objects | margin dB (20 log10 of",
        "# the side-lobe floor over the weakest object; floor = largest |A| beyond +-3 cells of",
        "# every object) | each object's level over the floor, dB, targets then clutter.",
    ]
    for scene, noise, res in rows():
        for surf in SURFACES:
            lines.append(format_row(scene, noise, surf, res[surf]))
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
