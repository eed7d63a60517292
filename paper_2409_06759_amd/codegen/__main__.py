"""Print the derived equations: python -m paper_2409_06759_amd.codegen ccsd"""
import sys

from . import equations
from .diagrams import diagram_count


def main(argv=None):
    method = (argv or sys.argv[1:] or ["ccsd"])[0]
    eq = equations(method)
    print(f"# {method.upper()}: {diagram_count(method)} diagrams")
    for k, terms in eq.items():
        print(f"## {'energy' if k == 0 else f'R{k}'}: {len(terms)} terms")
        for t in terms:
            print(f"{str(t.diagram.string()):40s} {t.text()}")


if __name__ == "__main__":
    main()
