"""MI355X-native FireANTs dense matching step (placeholder; binding added below)."""
