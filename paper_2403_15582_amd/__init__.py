"""MI355X-native multi-tone additive synthesis (placeholder, binding added below)."""
