"""CPU oracle of the periodic adjoint method (test infrastructure only)."""
