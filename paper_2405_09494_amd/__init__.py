"""MI355X-native symmetry-adapted finite-temperature GW hot path (libgwsym + binding)."""
