"""MI355X-native patch-group MUSCL-Hancock Euler solver (GAMER-2 hot path)."""
