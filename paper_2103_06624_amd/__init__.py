"""MI355X-native beta-CROWN bound propagation (libcvbound + a thin binding)."""
