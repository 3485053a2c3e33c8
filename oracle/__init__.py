"""FP64 CPU oracle of the IBM-HT step. Test infrastructure only (see oracle.py)."""
