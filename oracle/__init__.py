"""CPU oracle (test infrastructure only): see gao.h."""
