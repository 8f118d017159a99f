"""MI355X-native QED Monte-Carlo photon emission and pair production step."""
