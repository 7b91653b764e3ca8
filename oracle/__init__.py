"""CPU oracle of the bulb-model flavor evolution -- test infrastructure only."""
