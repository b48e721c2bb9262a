"""CPU oracle of the IPC Newton step (test infrastructure only; see ref.py)."""
