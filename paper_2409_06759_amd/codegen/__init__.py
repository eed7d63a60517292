"""Diagrammatic derivation of the coupled-cluster amplitude equations.

Distinct Kucharski-Bartlett diagrams are enumerated from integer triples in
the spirit of the string representation of Kallay and Surjan (paper, Sec.
"Coupled cluster amplitude equations", Fig. "algo:gen"), turned into
directed line graphs, and interpreted into explicit tensor terms with the
usual Goldstone rules (sign from hole lines and loops, weights from
equivalent lines and vertices, antisymmetrisers over inequivalent external
lines).  The derivation is host-side Python.
"""
from .diagrams import Diagram, HPiece, TVertex, diagram_count, enumerate_diagrams, method_diagrams
from .terms import Term, interpret, equations

__all__ = ["Diagram", "HPiece", "TVertex", "diagram_count", "enumerate_diagrams", "method_diagrams", "Term",
           "interpret", "equations"]
