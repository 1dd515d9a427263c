"""Generate the per-process HIP headers: python -m paper_2510_05100_amd.procgen OUTDIR"""
import os
import sys

from . import diagrams, emit

PROCESSES = {
    "ee_mumu": "e+ e- > mu+ mu-",
    "uu_eeg": "u u~ > e+ e- g",
    "gg_ttgg": "g g > t t~ g g",
    "gg_tttt": "g g > t t~ t t~",
}


def main(outdir):
    os.makedirs(outdir, exist_ok=True)
    for name, text in PROCESSES.items():
        d = diagrams.build(diagrams.parse(name, text))
        src = emit.generate(d)
        path = os.path.join(outdir, f"gen_{name}.h")
        old = open(path).read() if os.path.exists(path) else None
        if old != src:
            with open(path, "w") as f:
                f.write(src)
        print(f"{name}: {d.n_diagrams} diagrams, {len(d.terms)} amplitude terms, {len(d.basis)} colour flows -> {path}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__), "..", "csrc", "generated"))
