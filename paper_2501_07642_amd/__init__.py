"""MI355X-native rerandomization hot path (placeholder; the binding is added with the library)."""
